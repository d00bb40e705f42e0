"""Parity at the full workload sizes, in the launch configuration the bench
times: the whole batch runs on the GPU and the oracle checks a seeded sample
of the results one by one, or properties that hold at any size.

* 8-qubit noisy QAOA, 1024 parameter sets x 1000 chains, 10 burn-in sweeps:
  chi-square of sampled parameter sets against the density-matrix diagonal
  (and uniform p-values across them), the MaxCut cost of every sample, and
  the score-function gradient over the sampled states against the oracle's
  product rule for sampled parameter sets, and sampled chains against the
  oracle's chain with the same random stream (the same final state wherever
  no decision is a near tie);
* 16-qubit p=2 noisy QAOA, 262,144 amplitudes: sampled rows against the
  oracle's branch amplitudes (complex128 amplitudes, complex64
  probabilities), every row's complex64 probability against complex128
  (1e-5 relative), the complex64 gradient against complex128;

The 8- and 16-qubit ACs come from the search-based compiler, as in the bench.
* 32-qubit noise-free QAOA, 256 x 3907 chains: per-edge <Z_i Z_j> of sampled
  parameter sets against the light cone, and every sample's cost.
"""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import gibbs
from oracle import grad as ograd
from oracle import sim, stats
from paper_2103_17226_amd.dnnf import compile_circuit_dpll
from tests.gpu_common import graph, note, oracle_amplitudes, prob_ok, require_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _gpu():
    require_gpu()


def _bits(x, n):
    x = np.asarray(x).reshape(-1).view(np.uint64)
    return ((x[:, None] >> np.arange(n, dtype=np.uint64)) & np.uint64(1)).astype(np.int64)


def test_config2_full_batch_samples_costs_and_gradient():
    cfg = W.config(2)
    circ = cfg["circuit"]
    theta = cfg["theta"]
    P, C = theta.shape[0], cfg["chains_per_param"]
    note(f"config 2 full batch: {P} x {C} chains")
    g = graph(compile_circuit_dpll(circ))            # the AC the bench runs
    out = g.sample(theta, C, 1, 10, 1, 2024, cost_edges=circ.edges, dtype="c64", want_states=True,
                   want_cost=True, validate=False)
    x = out["samples"].cpu().numpy().reshape(P, C)
    cost = out["cost"].cpu().numpy().reshape(P, C)
    bits = _bits(x, circ.n)
    assert np.array_equal(cost.reshape(-1), W.maxcut_cost(circ.edges, bits).astype(np.float64))
    rng = np.random.default_rng(3)
    pick = np.sort(rng.choice(P, size=24, replace=False))
    pvals = []
    for p in pick:
        probs = sim.probabilities(circ, theta[p])
        _, _, pv = stats.chi2_pooled(np.bincount(x[p].astype(np.int64), minlength=1 << circ.n), probs)
        pvals.append(pv)
    note(f"  chi2 p-values: min {min(pvals):.3g}, KS {stats.uniformity_pvalue(pvals):.3g}")
    assert min(pvals) > 1e-5
    assert stats.uniformity_pvalue(pvals) > 1e-3
    # the bench's gradient: LOGPROB over the sampled states, weight = cost
    states = out["states"].reshape(P * C, -1)
    po = torch.arange(P, dtype=torch.int32, device=states.device).repeat_interleave(C)
    grad = g.grad(theta, states, po, mode="logprob", weight=out["cost"].reshape(-1), dtype="c64",
                  validate=False)["grad"].cpu().numpy()
    vals = W.unpack_evidence(circ, states.cpu().numpy().view(np.uint64))
    for p in pick[:2]:
        want = np.zeros(circ.n_angles)
        mass = np.zeros(circ.n_angles)          # sum of |terms|: the score terms cancel
        cache = {}
        for c in range(C):
            v = vals[p * C + c]
            k = tuple(int(z) for z in v[circ.n:])
            if k not in cache:
                kk = np.array(k)
                cache[k] = (sim.branch_state(circ, theta[p], kk), ograd.amplitude_grad(circ, theta[p], kk))
            psi, dpsi = cache[k]
            xi = sum(int(v[q]) << q for q in range(circ.n))
            f, df = psi[xi], dpsi[:, xi]
            if abs(f) > 0:
                term = cost[p, c] * 2.0 * np.real(np.conj(f) * df) / abs(f) ** 2
                want += term
                mass += np.abs(term)
        note(f"  param {p}: gradient {grad[p]} vs oracle {want} (term mass {mass})")
        assert np.all(np.abs(grad[p] - want) <= 1e-5 * mass)


def _oracle_chain_with_margin(circ, theta, seed, ch, sweeps):
    """The oracle's systematic-scan chain, and the smallest distance of any of
    its decisions' targets r * total from a cumulative-weight boundary,
    relative to the total."""
    bc = gibbs.BranchCache(circ, theta)
    s = gibbs.init_state(circ, seed, ch)
    margin = 1.0
    for sweep in range(sweeps):
        for v in range(circ.n_vars):
            w = gibbs.conditional_weights(bc, s, v)
            r = gibbs.uniform(seed, ch, sweep, v)
            u = gibbs.choose(w, r)
            if u is not None:
                s[v] = u
            tot = sum(w)
            if tot > 0:
                margin = min(margin, float(np.min(np.abs(r * tot - np.cumsum(w)))) / tot)
    return s, margin


def test_config2_full_batch_chains_follow_the_oracle_chain():
    """Sampled chains of the full batch, in complex64, against the oracle's
    complex128 chain with the same random stream.  A complex64 decision can
    differ from the oracle's only if the target r * total lies within the
    weights' rounding error of a cumulative boundary: |d|^2 from complex64
    derivatives is within ~6e-6 relative of complex128 (the measured
    branch-probability error), so a boundary and the target each move by at
    most ~6e-6 of the total.  Chains whose every decision is farther than
    5e-5 of the total from a boundary must end in the oracle's state
    exactly."""
    cfg = W.config(2)
    circ = cfg["circuit"]
    theta = cfg["theta"]
    P, C = theta.shape[0], cfg["chains_per_param"]
    seed, burn = 777, 10
    note(f"config 2 full batch, complex64 chains against the oracle chain: {P} x {C} chains")
    g = graph(compile_circuit_dpll(circ))            # the AC the bench runs
    out = g.sample(theta, C, 1, burn, 1, seed, dtype="c64", want_states=True, validate=False)
    states = out["states"].reshape(P * C, -1).cpu().numpy().view(np.uint64)
    rng = np.random.default_rng(11)
    chains = np.sort(rng.choice(P * C, size=6, replace=False))
    exact = 0
    for ch in chains:
        ref, margin = _oracle_chain_with_margin(circ, theta[ch // C], seed, int(ch), burn + 1)
        got = W.unpack_evidence(circ, states[ch])[0]
        same = np.array_equal(got, np.array(ref))
        note(f"  chain {ch}: {'same state' if same else 'differs'}, smallest decision margin {margin:.2e}")
        if margin > 5e-5:
            assert same, (int(ch), margin)
            exact += 1
    assert exact >= 3


def test_config3_full_batch_amplitudes_and_gradient():
    cfg = W.config(3)
    circ = cfg["circuit"]
    theta, ev, po = cfg["theta"], cfg["evidence"], cfg["param_of"]
    B = ev.shape[0]
    note(f"config 3 full batch: {B} amplitudes")
    g = graph(compile_circuit_dpll(circ))            # the AC the bench runs

    def free():
        g.release_workspaces()
        torch.cuda.empty_cache()

    a64, p64 = g.eval(theta, ev, po, dtype="c64", validate=False)
    free()
    a128, p128 = g.eval(theta, ev, po, dtype="c128", validate=False)
    free()
    a128 = a128.cpu().numpy()
    p64, p128 = p64.cpu().numpy(), p128.cpu().numpy()
    # every result: complex64 against complex128 (branch probabilities, 1e-5)
    ok, worst = prob_ok(p64, p128, rel=1e-5)
    note(f"  c64 vs c128 worst rel err {worst:.2e}")
    assert ok
    # sampled rows against the oracle's branch amplitudes
    vals = W.unpack_evidence(circ, ev)
    rng = np.random.default_rng(11)
    rows = np.sort(rng.choice(B, size=16, replace=False))
    ref = np.array([oracle_amplitudes(circ, theta[po[b]], vals[b:b + 1])[0] for b in rows])
    assert np.max(np.abs(a128[rows] - ref)) <= 1e-12
    ok, worst = prob_ok(p64[rows], np.abs(ref) ** 2)            # complex64 rows against the oracle itself
    note(f"  c64 sampled rows vs oracle worst rel err {worst:.2e}")
    assert ok
    # gradient of sum_b |f_b|^2 at full size: complex64 against complex128
    w = np.ones(B)
    g64 = g.grad(theta, ev, po, mode="prob", weight=w, dtype="c64", validate=False)["grad"].cpu().numpy()
    free()
    g128 = g.grad(theta, ev, po, mode="prob", weight=w, dtype="c128", validate=False)["grad"].cpu().numpy()
    free()
    scale = np.max(np.abs(g128))
    note(f"  gradient c64 vs c128: max |diff| / max |g| = {np.max(np.abs(g64 - g128)) / scale:.2e}")
    assert np.max(np.abs(g64 - g128)) <= 1e-4 * scale


def test_config4_full_batch_lightcone_and_costs():
    cfg = W.config(4)
    circ = cfg["circuit"]
    theta = cfg["theta"]
    P, C = theta.shape[0], cfg["chains_per_param"]
    note(f"config 4 full batch: {P} x {C} chains")
    g = graph(circ)
    out = g.sample(theta, C, 1, 10, 1, 77, cost_edges=circ.edges, dtype="c64", want_cost=True, validate=False)
    x = out["samples"].cpu().numpy().reshape(P, C)
    cost = out["cost"].cpu().numpy().reshape(P, C)
    assert np.array_equal(cost.reshape(-1), W.maxcut_cost(circ.edges, _bits(x, circ.n)).astype(np.float64))
    rng = np.random.default_rng(5)
    n_e = len(circ.edges)
    for p in rng.choice(P, size=4, replace=False):
        spins = 1 - 2 * _bits(x[p], circ.n)
        for (i, j) in circ.edges:
            est = float(np.mean(spins[:, i] * spins[:, j]))
            ref = sim.qaoa_p1_zz_lightcone(circ.edges, theta[p, 0], theta[p, 1], i, j)
            sd = np.sqrt(max(1.0 - ref * ref, 1e-3) / C)
            assert abs(est - ref) <= 5.0 * sd, (p, i, j, est, ref, n_e)
