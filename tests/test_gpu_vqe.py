"""The 2D Ising VQE workload on the same kernels: amplitudes, gradients and
samples against the oracle."""
import numpy as np
import pytest

import workloads as W
from oracle import grad as ograd
from oracle import sim, stats
from tests.gpu_common import graph, note, oracle_amplitudes, prob_ok, require_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _gpu():
    require_gpu()


def _noisy(p):
    edges, J, h = W.ising_instance(3, 3, W.sub_seed("graph", 6))
    return W.vqe_ising(3, 3, p, J, h, dep=0.005, ad=0.003)


def test_vqe_noisy_branch_amplitudes_c128_and_c64():
    circ = _noisy(2)
    note(f"vqe 3x3 p=2 noisy: {circ.n_vars} variables")
    g = graph(circ)
    rng = np.random.default_rng(1)
    P, B = 5, 300
    theta = rng.uniform(0, 2 * np.pi, size=(P, circ.n_angles))
    doms = circ.var_domains()
    vals = np.zeros((B, circ.n_vars), dtype=np.int64)
    vals[:, :circ.n] = rng.integers(0, 2, size=(B, circ.n))
    for v in range(circ.n, circ.n_vars):
        vals[:, v] = rng.integers(0, doms[v], size=B) * (rng.random(B) < 0.05)
    po = rng.integers(0, P, size=B).astype(np.int32)
    ev = W.pack_evidence(circ, vals)
    cache = {}
    ref = np.array([oracle_amplitudes(circ, theta[po[b]], vals[b:b + 1], cache)[0] for b in range(B)])
    amp, prob = g.eval(theta, ev, po, dtype="c128")
    assert np.max(np.abs(amp.cpu().numpy() - ref)) <= 1e-12
    amp64, prob64 = g.eval(theta, ev, po, dtype="c64")
    # branch probabilities (one Kraus branch, ~330 channel weights per
    # product) at the 1e-5 of the probability rule
    ok, rel = prob_ok(prob64.cpu().numpy(), np.abs(ref) ** 2, rel=1e-5)
    note(f"c64 branch probabilities: max rel {rel:.2e}")
    assert ok


def test_vqe_ideal_4x4_all_amplitudes():
    edges, J, h = W.ising_instance(4, 4, 11)
    circ = W.vqe_ising(4, 4, 2, J, h)
    note("vqe 4x4 p=2 ideal: all 65536 amplitudes")
    g = graph(circ)
    theta = np.array([[0.4, 1.1, 0.7, 2.0, 0.3, 1.4]])
    n = circ.n
    xs = np.arange(1 << n)
    bits = ((xs[:, None] >> np.arange(n)) & 1).astype(np.int64)
    ev = W.pack_evidence(circ, bits)
    amp, prob = g.eval(theta, ev, np.zeros(len(xs), np.int32), dtype="c128")
    psi = sim.statevector(circ, theta[0])
    assert np.max(np.abs(amp.cpu().numpy() - psi)) <= 1e-12
    assert abs(float(prob.sum().item()) - 1.0) < 1e-12


def test_vqe_gradient_matches_product_rule_and_finite_differences():
    # couplings and fields of both signs give angle gates with negative scales
    circ = _noisy(1)
    note("vqe gradients")
    g = graph(circ)
    rng = np.random.default_rng(4)
    theta = rng.uniform(0, 2 * np.pi, size=circ.n_angles)
    B = 40
    doms = circ.var_domains()
    vals = np.zeros((B, circ.n_vars), dtype=np.int64)
    vals[:, :circ.n] = rng.integers(0, 2, size=(B, circ.n))
    for v in range(circ.n, circ.n_vars):
        vals[:, v] = rng.integers(0, doms[v], size=B) * (rng.random(B) < 0.1)
    ev = W.pack_evidence(circ, vals)
    out = g.grad(theta[None, :], ev, None, mode="cotangent", cotangent=np.ones(B, dtype=np.complex128),
                 dtype="c128", want_dfdtheta=True)
    d = out["dfdtheta"].cpu().numpy()
    for b in range(0, B, 7):
        x = sum(int(vals[b, q]) << q for q in range(circ.n))
        want = ograd.amplitude_grad(circ, theta, vals[b, circ.n:])[:, x]
        assert np.max(np.abs(d[b] - want)) <= 1e-11
    # the energy-weighted loss L = sum_b E(x_b) |f_b|^2: GPU gradient vs central differences of the oracle
    w = W.ising_energy(circ.edges, circ.couplings, circ.fields, vals[:, :circ.n])
    gpu = g.grad(theta[None, :], ev, None, mode="prob", weight=w, dtype="c128")["grad"].cpu().numpy()[0]

    def loss(th):
        cache = {}
        f = np.array([oracle_amplitudes(circ, th, vals[b:b + 1], cache)[0] for b in range(B)])
        return float(np.dot(w, np.abs(f) ** 2))

    fd = ograd.central_difference(loss, theta, 1e-6)
    assert np.allclose(gpu, fd, rtol=1e-6, atol=1e-8 * max(1.0, np.max(np.abs(fd))))


def test_vqe_noisy_samples_chi2_against_density_matrix():
    circ = _noisy(1)
    note("vqe sampling vs density matrix")
    g = graph(circ)
    theta = np.array([[0.9, 0.4, 1.2]])
    C = 30000
    out = g.sample(theta, C, 1, 25, 1, 2024, dtype="c64")
    x = out["samples"].cpu().numpy().reshape(-1).view(np.uint64).astype(np.int64)
    counts = np.bincount(x, minlength=1 << circ.n).astype(float)
    p = sim.probabilities(circ, theta[0])
    _, _, pval = stats.chi2_pooled(counts, p / p.sum())
    note(f"chi2 p-value {pval:.3g}")
    assert pval > 1e-4
