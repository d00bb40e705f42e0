"""GPU parity of the Gibbs sampler (ac_sample).

* same chain, bit for bit: the oracle's reference chain (branch state
  vectors, the same counter-based SplitMix64 stream) and the GPU chain make
  the same decisions in complex128;
* finite-step law: histograms after t sweeps against the exact t-sweep
  distribution from explicit transition matrices (chi-square);
* stationary law: output histograms against the density-matrix diagonal.
"""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import gibbs, sim, stats
from tests.gpu_common import graph, note, require_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _gpu():
    require_gpu()


@pytest.mark.parametrize("variant", ["auto", "stream", "lds-cpw1", "lds-cpw2", "lds-cpw4", "global"])
def test_same_chain_bitwise_c128(variant, monkeypatch):
    note(f"same-chain bitwise ({variant})")
    if variant in ("global", "stream"):
        monkeypatch.setenv("QKC_SAMPLE_KERNEL", variant)
    elif variant != "auto":
        monkeypatch.setenv("QKC_SAMPLE_KERNEL", "lds")
        monkeypatch.setenv("QKC_SAMPLE_CPW", variant[-1])
    circ = W.qaoa_maxcut(3, W.ring_graph(3), 1, dep=0.05, ad=0.03)
    g = graph(circ)
    theta = np.array([[0.7, 0.4], [2.2, 1.3]])
    cpp, spc, burn, thin, seed = 3, 2, 3, 2, 12345
    out = g.sample(theta, cpp, spc, burn, thin, seed, dtype="c128", want_states=True, want_rounds=True)
    states = out["states"].cpu().numpy().view(np.uint64)
    samples = out["samples"].cpu().numpy().view(np.uint64)
    for p in range(2):
        for c in range(cpp):
            ch = p * cpp + c
            ref, _ = gibbs.run_chain(circ, theta[p], seed, ch, burn, thin, spc)
            for j in range(spc):
                got = W.unpack_evidence(circ, states[p, c * spc + j])[0]
                assert np.array_equal(got, ref[j]), (p, c, j)
                assert int(samples[p, c * spc + j, 0]) == W.x_index(ref[j][:circ.n])
    assert int(out["rounds"].min()) >= 1


@pytest.mark.parametrize("name,sweeps", [("ring3", 1), ("ring3", 2), ("bell", 1), ("bell", 3)])
def test_finite_sweep_distribution(name, sweeps):
    note(f"t-sweep law {name} t={sweeps}")
    if name == "bell":
        circ = W.noisy_bell(0.36)
        theta = np.zeros((1, 0))
    else:
        circ = W.qaoa_maxcut(3, W.ring_graph(3), 1)
        theta = np.array([[0.6, 0.35]])
    g = graph(circ)
    states, dist = gibbs.exact_sweep_distribution(circ, theta[0], sweeps)
    chains = 40000
    out = g.sample(theta, chains, 1, sweeps - 1, 1, seed=99 + sweeps, dtype="c64", want_states=True)
    st = W.unpack_evidence(circ, out["states"].cpu().numpy().reshape(-1, circ.n_words).view(np.uint64))
    index = {tuple(s): i for i, s in enumerate(states.tolist())}
    counts = np.zeros(len(states))
    for s in st.tolist():
        counts[index[tuple(s)]] += 1
    _, _, pval = stats.chi2_pooled(counts, dist)
    note(f"  p = {pval:.3g}")
    assert pval > 1e-4


def test_stationary_distribution_noisy_qaoa_n8():
    note("stationary law vs density matrix, noisy n=8")
    cfg = W.config(2, small=True)
    circ = cfg["circuit"]
    g = graph(circ)
    P, chains, burn = 4, 4000, 40
    theta = cfg["theta"][:P]
    out = g.sample(theta, chains, 1, burn, 1, seed=2024, dtype="c64", want_rounds=True)
    x = out["samples"].cpu().numpy().reshape(P, chains)
    pvals = []
    for p in range(P):
        probs = sim.probabilities(circ, theta[p])
        counts = np.bincount(x[p], minlength=1 << circ.n)
        _, _, pv = stats.chi2_pooled(counts, probs)
        pvals.append(pv)
        note(f"  param {p}: p = {pv:.3g}, KL = {stats.kl_divergence(counts, probs):.3g}")
    note(f"  mean rounds per chain {out['rounds'].double().mean().item():.1f}")
    assert min(pvals) > 1e-4


@pytest.mark.parametrize("other", ["lds", "global", "auto"])
def test_sampler_kernels_agree_c128(other, monkeypatch):
    note(f"streaming sampler kernel vs {other}")
    cfg = W.config(2, small=True)
    g = graph(cfg["circuit"])
    theta = cfg["theta"][:3]
    kw = dict(chains_per_param=40, samples_per_chain=2, burn_in=3, thin=1, seed=11, dtype="c128",
              want_states=True, want_rounds=True)
    monkeypatch.setenv("QKC_SAMPLE_KERNEL", "stream")
    a = g.sample(theta, **kw)
    if other == "auto":
        monkeypatch.delenv("QKC_SAMPLE_KERNEL")
    else:
        monkeypatch.setenv("QKC_SAMPLE_KERNEL", other)
    b = g.sample(theta, **kw)
    assert torch.equal(a["states"], b["states"]) and torch.equal(a["rounds"], b["rounds"])


def test_sampler_determinism_and_cost():
    note("determinism and cost")
    cfg = W.config(2, small=True)
    circ = cfg["circuit"]
    g = graph(circ)
    theta = cfg["theta"][:3]
    kw = dict(chains_per_param=70, samples_per_chain=3, burn_in=4, thin=2, cost_edges=circ.edges,
              want_cost=True, want_states=True)
    a = g.sample(theta, seed=5, **kw)
    b = g.sample(theta, seed=5, **kw)
    c = g.sample(theta, seed=6, **kw)
    assert torch.equal(a["samples"], b["samples"]) and torch.equal(a["states"], b["states"])
    assert not torch.equal(a["samples"], c["samples"])
    x = a["samples"].cpu().numpy().reshape(-1).view(np.uint64)
    bits = np.array([W.x_bits(int(v), circ.n) for v in x])
    assert np.array_equal(a["cost"].cpu().numpy().reshape(-1), W.maxcut_cost(circ.edges, bits))
