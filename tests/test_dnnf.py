"""CPU checks of the search-based compiler (exhaustive DPLL with components,
caching and a dtree, Sec. 3.2.2) against the oracle: amplitudes on every
assignment, the multilinear polynomial in random indicators, the structural
properties that make the AC a smooth decomposable circuit, and its sizes next
to the paper's Table variational_problem_size_metrics."""
import itertools

import numpy as np
import pytest

import workloads as W
from oracle import sim
from paper_2103_17226_amd import compiler as C
from paper_2103_17226_amd import cpu_eval
from paper_2103_17226_amd import dnnf as D
from paper_2103_17226_amd.blob import compile_blob, to_blob
from tests import ac_host_eval as H
from tests.test_compiler import CIRCUITS, all_assignments, oracle_amp


@pytest.mark.parametrize("dtree", ["order", "bisect"])
@pytest.mark.parametrize("selectors", [True, False])
@pytest.mark.parametrize("name", sorted(CIRCUITS))
def test_dpll_ac_matches_oracle_on_every_assignment(name, selectors, dtree):
    circ = CIRCUITS[name]()
    ac = D.compile_circuit_dpll(circ, selectors=selectors, dtree=dtree)
    rng = np.random.default_rng(3)
    theta = rng.uniform(0, 2 * np.pi, size=circ.n_angles)
    for vals in all_assignments(circ):
        assert abs(H.evaluate_assignment(ac, theta, vals) - oracle_amp(circ, theta, vals)) < 1e-13, vals


@pytest.mark.parametrize("dtree", ["order", "bisect"])
@pytest.mark.parametrize("selectors", [True, False])
@pytest.mark.parametrize("name", ["bell", "tiny", "ring3_dep"])
def test_dpll_ac_is_the_network_polynomial(name, selectors, dtree):
    # Smooth and multilinear: AC(lambda) = sum_s f(s) prod_v lambda_{v, s_v}
    # with the oracle's f, for indicators drawn at random
    circ = CIRCUITS[name]()
    ac = D.compile_circuit_dpll(circ, selectors=selectors, dtree=dtree)
    rng = np.random.default_rng(5)
    theta = rng.uniform(0, 2 * np.pi, size=circ.n_angles)
    doms = circ.var_domains()
    lam = [rng.normal(size=d) + 1j * rng.normal(size=d) for d in doms]
    expect = 0j
    for s in itertools.product(*[range(d) for d in doms]):
        expect += np.prod([lam[v][u] for v, u in enumerate(s)]) * oracle_amp(circ, theta, list(s))
    got = H.evaluate(ac, theta, lam)
    assert abs(got - expect) < 1e-12 * max(1.0, abs(expect))


def _child_evidence(ac):
    """Per internal node, the evidence variables each child's sub-circuit
    mentions (indicators, and the event variable of selector leaves)."""
    sel_var = [int(s[0]) for s in ac.selectors]
    mask = (1 << C.TAG_SHIFT) - 1
    below, kids = [], []
    for n in range(ac.n_internal):
        ks = []
        for r in ac.col[ac.row_ptr[n]:ac.row_ptr[n + 1]]:
            tag, idx = int(r) >> C.TAG_SHIFT, int(r) & mask
            if tag == C.TAG_NODE:
                ks.append(below[idx])
            elif tag == C.TAG_IND:
                ks.append(frozenset([idx & ((1 << C.IND_VAL_SHIFT) - 1)]))
            elif tag == C.TAG_SEL:
                ks.append(frozenset([sel_var[idx]]))
            else:
                ks.append(frozenset())
        kids.append(ks)
        below.append(frozenset().union(*ks))
    return below, kids


@pytest.mark.parametrize("name", ["tiny", "ring3_dep_ad", "vqe2x2_dep_ad", "vqe2x3_p2"])
def test_dpll_ac_is_decomposable_and_smooth(name):
    # products join children over disjoint evidence variables; the branches
    # of a sum mention the same evidence variables (flattening merges chains
    # of equal ops, which keeps both properties)
    circ = CIRCUITS[name]()
    ac = D.compile_circuit_dpll(circ)
    below, kids = _child_evidence(ac)
    for n in range(ac.n_internal):
        if ac.op[n] == C.OP_PROD:
            seen = set()
            for s in kids[n]:
                assert not (seen & s), n
                seen |= s
        else:
            assert all(s == kids[n][0] for s in kids[n]), n
    assert below[ac.root] == frozenset(range(len(circ.var_domains())))


def test_dtrees_cover_every_factor_once():
    circ = W.config(2, small=True)["circuit"]
    F = C.build_factors(circ)
    scopes = [f.vars for f in F.live]
    for root in (D.dtree_bisect(scopes), D.dtree_from_order(scopes, C._elimination_order(F.live, F.dom))):
        leaves = []
        stack = [root]
        while stack:
            t = stack.pop()
            if t.left is None:
                leaves.extend(t.factors)
                continue
            assert t.factors == t.left.factors | t.right.factors
            assert not (t.left.factors & t.right.factors)
            vl = {v for f in t.left.factors for v in scopes[f]}
            vr = {v for f in t.right.factors for v in scopes[f]}
            assert set(t.cut) == vl & vr
            stack += [t.left, t.right]
        assert sorted(leaves) == list(range(len(scopes)))


def test_bisection_keeps_halves_balanced_and_cuts_few_variables():
    # a chain of factors (v_i, v_i+1) splits into two runs sharing one variable
    scopes = [(i, i + 1) for i in range(40)]
    a, b = D._bisect(list(range(40)), scopes)
    assert 16 <= len(a) <= 24
    va = {v for f in a for v in scopes[f]}
    vb = {v for f in b for v in scopes[f]}
    assert len(va & vb) == 1


@pytest.mark.parametrize("seed", [1, 2, 3, 4, 5, 6])
def test_dpll_random_circuits_through_the_blob_and_cpu_evaluator(seed):
    circ = W.random_circuit(seed)
    cpu = cpu_eval.CpuAC(compile_blob(circ, method="dpll"))
    rng = np.random.default_rng(seed)
    theta = rng.uniform(-3, 3, size=(2, circ.n_angles))
    doms = circ.var_domains()
    vals = np.array([[int(rng.integers(0, d)) for d in doms] for _ in range(40)], dtype=np.int64)
    po = (np.arange(40) % 2).astype(np.int32)
    amp = cpu.eval(theta, W.pack_evidence(circ, vals), po, threads=2)
    for b in range(40):
        x = sum(int(vals[b, q]) << q for q in range(circ.n))
        ref = sim.amplitude(circ, theta[po[b]], x, vals[b, circ.n:])
        assert abs(amp[b] - ref) <= 1e-12, (seed, b)


# The noisy rows of Table variational_problem_size_metrics (depolarizing 0.5%
# after every gate): AC nodes of the paper's compiler on its instances.  Ours
# are on seeded instances of the same shapes, so only the order is compared.
PAPER_NOISY = {
    "qaoa12_p1": (lambda: W.qaoa_maxcut(12, W.random_regular_graph(12, 3, 11), 1, dep=0.005), 5798),
    "vqe9_p1": (lambda: W.vqe_ising(3, 3, 1, *W.ising_instance(3, 3, 3)[1:], dep=0.005), 3810),
    "vqe9_p2": (lambda: W.vqe_ising(3, 3, 2, *W.ising_instance(3, 3, 3)[1:], dep=0.005), 7701),
}


@pytest.mark.parametrize("name", sorted(PAPER_NOISY))
def test_dpll_sizes_are_of_the_papers_order(name):
    make, paper_nodes = PAPER_NOISY[name]
    circ = make()
    dp = D.compile_circuit_dpll(circ)
    ve = C.compile_circuit(circ)
    assert dp.n_internal <= 2 * paper_nodes
    assert dp.n_internal <= 1.5 * ve.n_internal
    rng = np.random.default_rng(8)
    theta = rng.uniform(0, 2 * np.pi, size=circ.n_angles)
    doms = circ.var_domains()
    for _ in range(6):
        vals = [int(rng.integers(0, 2)) for _ in range(circ.n)] + [0] * (len(doms) - circ.n)
        for v in rng.choice(np.arange(circ.n, len(doms)), size=2, replace=False):
            vals[int(v)] = int(rng.integers(0, doms[int(v)]))
        assert abs(H.evaluate_assignment(dp, theta, vals) - oracle_amp(circ, theta, vals)) < 1e-13


def test_dpll_blob_is_cached_under_its_own_key(tmp_path):
    from paper_2103_17226_amd.blob import compile_blob_cached
    circ = CIRCUITS["tiny"]()
    a, hit_a = compile_blob_cached(circ, str(tmp_path), method="dpll")
    b, hit_b = compile_blob_cached(circ, str(tmp_path))
    c, hit_c = compile_blob_cached(circ, str(tmp_path), method="dpll")
    assert (hit_a, hit_b, hit_c) == (False, False, True)
    assert a == c == to_blob(D.compile_circuit_dpll(circ)) and b == compile_blob(circ)
    with pytest.raises(ValueError):
        compile_blob(circ, method="nope")


MPE_CIRCUITS = ["bell", "tiny", "ring3_dep", 0, 1, 2, 3, 4, 7, 8, 11]


def _mpe_circuit(name):
    return CIRCUITS[name]() if name in CIRCUITS else W.random_circuit(name)


@pytest.mark.parametrize("name", MPE_CIRCUITS)
def test_mpe_compilation_gives_the_most_probable_events(name):
    # events decided first: max-product over the AC equals the oracle's
    # largest |f(x, k)|^2, and the events it reads off achieve it
    circ = _mpe_circuit(name)
    ac = D.compile_circuit_dpll(circ, mpe=True)
    assert not ac.selectors
    rng = np.random.default_rng(21)
    theta = rng.uniform(0, 2 * np.pi, size=circ.n_angles)
    for x in range(1 << circ.n):
        bits = [(x >> q) & 1 for q in range(circ.n)]
        best, ks = sim.most_probable_events(circ, theta, x)
        m, k = H.max_product(ac, theta, bits)
        assert abs(m - best) <= 1e-12 * max(best, 1e-300), (x, m, best)
        if best > 0:
            assert tuple(k) in ks, (x, k, ks)
    # the same AC still gives every amplitude
    for vals in all_assignments(circ)[:200]:
        assert abs(H.evaluate_assignment(ac, theta, vals) - oracle_amp(circ, theta, vals)) < 1e-13


def test_best_of_both_compilers_is_the_smaller_ac():
    from paper_2103_17226_amd.blob import blob_summary
    for circ in (W.config(2, small=True)["circuit"], CIRCUITS["vqe2x2_dep_ad"]()):
        sizes = {m: blob_summary(compile_blob(circ, method=m))["n_int"] for m in ("ve", "dpll", "best")}
        assert sizes["best"] == min(sizes["ve"], sizes["dpll"])
