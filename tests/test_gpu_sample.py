"""GPU parity of the Gibbs sampler (ac_sample).

* same chain, bit for bit: the oracle's reference chain (branch state
  vectors, the same counter-based SplitMix64 stream) and the GPU chain make
  the same decisions in complex128;
* finite-step law: histograms after t sweeps against the exact t-sweep
  distribution from explicit transition matrices (chi-square);
* stationary law: output histograms against the density-matrix diagonal.
"""
import itertools

import numpy as np
import pytest
import torch

import workloads as W
from oracle import gibbs, sim, stats
from paper_2103_17226_amd.dnnf import compile_circuit_dpll
from tests.gpu_common import graph, note, require_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _gpu():
    require_gpu()


def oracle_changes(circ, theta, seed, chain, sweeps):
    """(visits of the oracle's chain that change its state, whether the last
    visit is one of them), from the oracle's own per-visit steps."""
    bc = gibbs.BranchCache(circ, theta)
    s = gibbs.init_state(circ, seed, chain)
    n, last = 0, False
    for sw in range(sweeps):
        for v in range(circ.n_vars):
            u = gibbs.choose(gibbs.conditional_weights(bc, s, v), gibbs.uniform(seed, chain, sw, v))
            last = u is not None and u != s[v]
            if last:
                s[v] = u
                n += 1
    return n, last


@pytest.mark.parametrize("variant", ["auto", "stream", "stream-sib3", "lds-cpw1", "lds-cpw2", "lds-cpw4", "lds-wpc4",
                                     "global"])
def test_same_chain_bitwise_c128(variant, monkeypatch):
    note(f"same-chain bitwise ({variant})")
    if variant in ("global", "stream"):
        monkeypatch.setenv("QKC_SAMPLE_KERNEL", variant)
    elif variant == "stream-sib3":                   # three-sibling occurrence groups
        monkeypatch.setenv("QKC_SAMPLE_KERNEL", "stream")
        monkeypatch.setenv("QKC_SAMPLE_SIB3", "1")
    elif variant == "lds-wpc4":                      # four waves on each chain
        monkeypatch.setenv("QKC_SAMPLE_KERNEL", "lds")
        monkeypatch.setenv("QKC_SAMPLE_CPW", "1")
        monkeypatch.setenv("QKC_SAMPLE_WPC", "4")
    elif variant != "auto":
        monkeypatch.setenv("QKC_SAMPLE_KERNEL", "lds")
        monkeypatch.setenv("QKC_SAMPLE_CPW", variant[-1])
        monkeypatch.setenv("QKC_SAMPLE_WPC", "1")
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
    # derivatives are reused while the state is unchanged: one upward and
    # downward pass per change, plus one for the visits after the last change
    rounds = out["rounds"].cpu().numpy()
    visits = 0
    for p in range(2):
        for c in range(cpp):
            ch = p * cpp + c
            n, last = oracle_changes(circ, theta[p], seed, ch, burn + spc * thin)
            assert int(rounds[ch]) == n + (0 if last else 1), (ch, int(rounds[ch]), n, last)
            visits += (burn + spc * thin) * circ.n_vars
    assert rounds.sum() < visits


def test_two_sibling_groups_give_the_same_chains(monkeypatch):
    # the streaming sampler takes larger occurrence groups when no occurrence
    # of the plan has a third sibling; the terms are added in the same order,
    # so the chains equal those of the three-sibling groups bit for bit
    monkeypatch.setenv("QKC_SAMPLE_KERNEL", "stream")
    cfg = W.config(2)
    circ = cfg["circuit"]
    outs = []
    for forced in ("0", "1"):
        monkeypatch.setenv("QKC_SAMPLE_SIB3", forced)
        g = graph(compile_circuit_dpll(circ))
        if forced == "0":
            assert g.info["max_siblings"] == 2
        for dtype in ("c64", "c128"):
            out = g.sample(cfg["theta"][:8], 300, 1, 4, 1, 5, dtype=dtype, want_states=True, want_rounds=True)
            outs.append((out["states"].cpu(), out["rounds"].cpu()))
    for a, b in zip(outs[:2], outs[2:]):
        assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])
    # plans with a third sibling exist among the test circuits (they run the
    # three-sibling groups: test_gpu_random_circuits, and the stream-sib3
    # variant of test_same_chain_bitwise_c128 forces them)
    monkeypatch.delenv("QKC_SAMPLE_SIB3")
    sibs = [graph(W.random_circuit(k)).info["max_siblings"] for k in range(6)]
    note(f"  most siblings of random circuits 0-5: {sibs}")
    assert 3 in sibs and all(0 <= x <= 3 for x in sibs)


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


@pytest.mark.parametrize("other", ["lds", "lds-wpc4", "global", "auto"])
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
    elif other == "lds-wpc4":
        monkeypatch.setenv("QKC_SAMPLE_KERNEL", "lds")
        monkeypatch.setenv("QKC_SAMPLE_CPW", "1")
        monkeypatch.setenv("QKC_SAMPLE_WPC", "4")
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


@pytest.mark.parametrize("variant", ["stream", "lds", "global"])
@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_resumed_chains_continue_one_long_run(variant, dtype, monkeypatch):
    # Two calls, the second started from the first call's last states with
    # first_sweep advanced, reproduce the later samples of one longer call.
    note(f"resumed chains ({variant}, {dtype})")
    monkeypatch.setenv("QKC_SAMPLE_KERNEL", variant)
    cfg = W.config(2, small=True)
    g = graph(cfg["circuit"])
    theta = cfg["theta"][:3]
    P, C = theta.shape[0], 40
    common = dict(chains_per_param=C, burn_in=3, thin=2, seed=77, dtype=dtype, want_states=True)
    whole = g.sample(theta, samples_per_chain=4, **common)
    first = g.sample(theta, samples_per_chain=2, **common)
    Wn = g.info["n_words"]
    st1 = first["states"].reshape(P, C, 2, Wn)
    assert torch.equal(st1, whole["states"].reshape(P, C, 4, Wn)[:, :, :2])
    last = st1[:, :, 1].reshape(P * C, Wn)
    second = g.sample(theta, chains_per_param=C, samples_per_chain=2, burn_in=0, thin=2, seed=77, dtype=dtype,
                      want_states=True, init_states=last, first_sweep=3 + 2 * 2)
    want = whole["states"].reshape(P, C, 4, Wn)[:, :, 2:]
    assert torch.equal(second["states"].reshape(P, C, 2, Wn), want)
    assert torch.equal(second["samples"].reshape(P, C, 2, -1), whole["samples"].reshape(P, C, 4, -1)[:, :, 2:])


def test_resumed_chains_from_arbitrary_states_follow_the_oracle_chain():
    # A chain started from a given state makes the oracle's decisions from that state.
    note("warm start vs oracle chain")
    circ = W.qaoa_maxcut(3, W.ring_graph(3), 1, dep=0.05, ad=0.03)
    g = graph(circ)
    theta = np.array([[0.7, 0.4]])
    rng = np.random.default_rng(3)
    doms = circ.var_domains()
    C = 6
    vals = np.stack([[rng.integers(0, d) for d in doms] for _ in range(C)])
    init = W.pack_evidence(circ, vals)
    out = g.sample(theta, C, 1, 2, 1, 99, dtype="c128", want_states=True, init_states=init, first_sweep=5)
    got = W.unpack_evidence(circ, out["states"].cpu().numpy().reshape(C, -1).view(np.uint64))
    for c in range(C):
        ref, _ = gibbs.run_chain(circ, theta[0], seed=99, chain=c, burn_in=2, thin=1, n_samples=1,
                                 init=vals[c], first_sweep=5)
        assert np.array_equal(got[c], ref[0]), c


def _posterior_circuit():
    return W.Circuit(n=2, ops=[("H", 0), ("DEP", 0, 0), ("H", 1), ("CNOT", 0, 1), ("AD", 1, 1),
                               ("RX", 0, 1, 2.0), ("RZ", 1, 0, 2.0), ("DEP", 1, 0)],
                     n_angles=2, noise=[0.3, 0.25], edges=[(0, 1)])


@pytest.mark.parametrize("variant", ["stream", "lds", "lds-wpc4", "global"])
def test_conditional_chains_follow_the_oracle_chain(variant, monkeypatch):
    # outputs held at an observed x (first_var = n): same decisions as the oracle
    note(f"conditional chains ({variant})")
    monkeypatch.setenv("QKC_SAMPLE_KERNEL", variant.split("-")[0])
    if variant == "lds-wpc4":
        monkeypatch.setenv("QKC_SAMPLE_CPW", "1")
        monkeypatch.setenv("QKC_SAMPLE_WPC", "4")
    circ = W.qaoa_maxcut(3, W.ring_graph(3), 1, dep=0.05, ad=0.03)
    g = graph(circ)
    theta = np.array([[0.7, 0.4]])
    C = 8
    vals = np.zeros((C, circ.n_vars), dtype=np.int64)
    vals[:, :circ.n] = [1, 0, 1]
    init = W.pack_evidence(circ, vals)
    out = g.sample(theta, C, 2, 3, 2, 5, dtype="c128", want_states=True, init_states=init, first_var=circ.n)
    got = W.unpack_evidence(circ, out["states"].cpu().numpy().reshape(C * 2, -1).view(np.uint64))
    for c in range(C):
        ref, _ = gibbs.run_chain(circ, theta[0], seed=5, chain=c, burn_in=3, thin=2, n_samples=2,
                                 init=vals[c], first_var=circ.n)
        assert np.array_equal(got[2 * c:2 * c + 2], ref), c


def test_error_posterior_and_most_probable_explanation():
    # noise events given an observed outcome: histogram vs |f(x, k)|^2 / sum_k,
    # and the most frequent event assignment is the exact MPE
    note("error posterior")
    circ = _posterior_circuit()
    g = graph(circ)
    th = np.array([[0.8, 1.3]])
    x = [1, 0]
    doms = circ.var_domains()[circ.n:]
    ks = list(itertools.product(*[range(d) for d in doms]))
    post = np.array([abs(sim.amplitude(circ, th[0], x[0] + 2 * x[1], k)) ** 2 for k in ks])
    post /= post.sum()
    C = 40000
    vals = np.zeros((C, circ.n_vars), dtype=np.int64)
    vals[:, :circ.n] = x
    out = g.sample(th, C, 1, 14, 1, 17, dtype="c64", want_states=True, init_states=W.pack_evidence(circ, vals),
                   first_var=circ.n)
    st = W.unpack_evidence(circ, out["states"].cpu().numpy().reshape(C, -1).view(np.uint64))
    assert np.all(st[:, :circ.n] == x)
    index = {k: i for i, k in enumerate(ks)}
    counts = np.zeros(len(ks))
    for row in st[:, circ.n:]:
        counts[index[tuple(int(v) for v in row)]] += 1
    _, _, pval = stats.chi2_pooled(counts, post)
    assert pval > 1e-4
    assert int(np.argmax(counts)) == int(np.argmax(post))


def _frozen_circuit():
    # RX(0) and RZ(0) leave |0..0>: every chain of outputs sits at x = 0 with
    # probability one after its first visit, so whole sweeps pass unchanged
    return W.Circuit(n=3, ops=[("RX", 0, 0, 1.0), ("CNOT", 0, 1), ("RX", 2, 0, 1.0), ("DEP", 1, 0),
                               ("RZ", 2, 1, 2.0)], n_angles=2, noise=[1e-9], edges=[(0, 1), (1, 2)])


@pytest.mark.parametrize("dtype", ["c64", "c128"])
@pytest.mark.parametrize("case", ["qaoa_n8", "random", "conditional", "frozen", "resumed"])
def test_decision_pass_matches_the_sequential_scan(case, dtype, monkeypatch):
    # The streaming sampler takes every variable's Gibbs choice for the round
    # in one pass over all waves and jumps to the first change; deciding each
    # visit in the scan instead must give the same chains, samples, costs and
    # round counts bit for bit (thinning, several samples per chain, held
    # variables, whole sweeps without a change, resumed chains).
    note(f"decision pass vs sequential scan ({case}, {dtype})")
    monkeypatch.setenv("QKC_SAMPLE_KERNEL", "stream")
    kw = dict(dtype=dtype, want_states=True, want_rounds=True)
    if case == "qaoa_n8":
        cfg = W.config(2, small=True)
        circ, theta = cfg["circuit"], cfg["theta"][:5]
        args = dict(chains_per_param=150, samples_per_chain=3, burn_in=4, thin=2, seed=21)
    elif case == "random":
        circ = W.random_circuit(8, n=5, n_ops=40)
        theta = np.random.default_rng(8).uniform(-3, 3, size=(3, circ.n_angles))
        args = dict(chains_per_param=100, samples_per_chain=2, burn_in=3, thin=1, seed=5)
    elif case == "conditional":
        circ = W.qaoa_maxcut(3, W.ring_graph(3), 1, dep=0.05, ad=0.03)
        theta = np.array([[0.7, 0.4], [1.9, 2.6]])
        vals = np.zeros((2 * 70, circ.n_vars), dtype=np.int64)
        vals[:, :circ.n] = [1, 0, 1]
        args = dict(chains_per_param=70, samples_per_chain=2, burn_in=2, thin=3, seed=6,
                    init_states=W.pack_evidence(circ, vals), first_var=circ.n)
    elif case == "frozen":
        circ = _frozen_circuit()
        theta = np.array([[0.0, 0.0], [1e-3, 0.0]])
        args = dict(chains_per_param=130, samples_per_chain=2, burn_in=3, thin=2, seed=9)
    else:
        cfg = W.config(2, small=True)
        circ, theta = cfg["circuit"], cfg["theta"][5:8]
        rng = np.random.default_rng(4)
        vals = np.stack([[rng.integers(0, d) for d in circ.var_domains()] for _ in range(3 * 64)])
        args = dict(chains_per_param=64, samples_per_chain=2, burn_in=1, thin=1, seed=13,
                    init_states=W.pack_evidence(circ, vals), first_sweep=17)
    g = graph(circ)
    if circ.edges:
        kw.update(cost_edges=circ.edges, want_cost=True)
    monkeypatch.setenv("QKC_SEQ_SCAN", "1")
    a = g.sample(theta, **args, **kw)
    monkeypatch.setenv("QKC_SEQ_SCAN", "0")
    b = g.sample(theta, **args, **kw)
    for key in ("samples", "states", "rounds") + (("cost",) if "cost_edges" in kw else ()):
        assert torch.equal(a[key], b[key]), key


@pytest.mark.parametrize("variant", ["stream", "lds", "global"])
@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_chain_offset_splits_a_request_exactly(variant, dtype, monkeypatch):
    # A request split by parameter sets (theta rows p0.., chain_offset =
    # p0 * chains_per_param) or by chains of one set (P = 1, chain_offset =
    # p * chains_per_param + c0) draws exactly the whole request's chains.
    note(f"chain offset ({variant}, {dtype})")
    monkeypatch.setenv("QKC_SAMPLE_KERNEL", variant)
    cfg = W.config(2, small=True)
    circ = cfg["circuit"]
    g = graph(circ)
    theta = cfg["theta"][:6]
    P, C = theta.shape[0], 50
    kw = dict(samples_per_chain=2, burn_in=3, thin=2, seed=31, dtype=dtype, cost_edges=circ.edges,
              want_states=True, want_cost=True, want_rounds=True)
    whole = g.sample(theta, C, **kw)
    Wn, S = g.info["n_words"], C * 2

    def part(p0, p1):
        return {k: whole[k].reshape(P, -1)[p0:p1] for k in ("samples", "states", "cost", "rounds")}
    for p0, p1 in ((0, 2), (2, 6)):
        got = g.sample(theta[p0:p1], C, chain_offset=p0 * C, **kw)
        want = part(p0, p1)
        for k in want:
            assert torch.equal(got[k].reshape(p1 - p0, -1), want[k]), (p0, k)
    p = 3
    for c0, c1 in ((0, 20), (20, 50)):
        got = g.sample(theta[p:p + 1], c1 - c0, chain_offset=p * C + c0, **kw)
        for k, per in (("samples", 2), ("states", 2 * Wn), ("cost", 2), ("rounds", 1)):
            flat = whole[k].reshape(P, C * per)[p]
            assert torch.equal(got[k].reshape(-1), flat[c0 * per:c1 * per]), (c0, k)


def test_cost_edges_outside_the_register_give_nan():
    note("cost edge outside the register")
    cfg = W.config(2, small=True)
    g = graph(cfg["circuit"])
    theta = cfg["theta"][:2]
    good = g.sample(theta, 64, seed=4, cost_edges=cfg["circuit"].edges, want_cost=True)
    bad = g.sample(theta, 64, seed=4, cost_edges=list(cfg["circuit"].edges) + [(0, 99)], want_cost=True,
                   validate=False)
    assert torch.equal(good["samples"], bad["samples"])
    assert torch.isnan(bad["cost"]).all()
