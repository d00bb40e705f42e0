"""CPU checks of the host compiler (circuit -> BN -> CNF -> AC -> blob).

Expected values come from the oracle (independent simulators), the paper's
printed BN sizes, or brute force; never from the GPU path.
"""
import itertools
import math
import struct

import numpy as np
import pytest

import workloads as W
from oracle import sim
from paper_2103_17226_amd import blob as blobmod
from paper_2103_17226_amd import compiler as C
from tests import ac_host_eval as H


def tiny_noisy():
    ops = [("H", 0), ("H", 1), ("CNOT", 0, 1), ("DEP", 1, 0), ("RZ", 1, 0, 2.0), ("AD", 0, 1),
           ("CNOT", 0, 1), ("RX", 0, 1, 2.0), ("PD", 1, 2), ("RX", 1, 1, 2.0), ("DEP", 0, 0)]
    return W.Circuit(n=2, ops=ops, n_angles=2, noise=[0.07, 0.2, 0.3], edges=[(0, 1)])


CIRCUITS = {
    "bell": lambda: W.noisy_bell(0.36),
    "tiny": tiny_noisy,
    "ring4": lambda: W.config(1, small=True)["circuit"],
    "ring3_dep_ad": lambda: W.qaoa_maxcut(3, W.ring_graph(3), 1, dep=0.05, ad=0.02),
    "vqe2x2_dep_ad": lambda: W.vqe_ising(2, 2, 1, [1.0, -1.0, -1.0, 1.0], [1.0, -1.0, 1.0, 1.0], dep=0.03, ad=0.02),
    "vqe2x3_p2": lambda: W.vqe_ising(2, 3, 2, *W.ising_instance(2, 3, 3)[1:]),
    "ring3_dep": lambda: W.Circuit(n=2, ops=[("H", 0), ("DEP", 0, 0), ("H", 1), ("CNOT", 0, 1), ("DEP", 1, 0), ("RZ", 1, 0, 2.0), ("DEP", 1, 0), ("CNOT", 0, 1), ("RX", 0, 1, 2.0), ("RX", 1, 1, 2.0), ("DEP", 0, 0)], n_angles=2, noise=[0.04], edges=[(0, 1)]),
}


def all_assignments(circ, limit=5000):
    doms = circ.var_domains()
    total = math.prod(doms)
    rng = np.random.default_rng(0)
    if total <= limit:
        return [list(a) for a in itertools.product(*[range(d) for d in doms])]
    return [[int(rng.integers(0, d)) for d in doms] for _ in range(limit // 10)]


def oracle_amp(circ, theta, values):
    n = circ.n
    x = sum(int(values[q]) << q for q in range(n))
    return sim.amplitude(circ, theta, x, values[n:])


# ------------------------------------------------------------------ BN / CNF

def test_bn_node_counts_match_paper_table():
    # Table variational_problem_size_metrics: ideal 32-qubit QAOA has 240 BN
    # nodes at one iteration and 416 at two (n initial states + one per gate)
    edges = W.random_regular_graph(32, 3, 11)
    for p, expect in ((1, 240), (2, 416)):
        bn = C.circuit_to_bn(W.qaoa_maxcut(32, edges, p))
        assert C.bn_node_count(bn) == expect


def test_bn_cats_are_transposed_gate_matrices():
    bn = C.circuit_to_bn(W.Circuit(n=1, ops=[("H", 0)], n_angles=0, noise=[]))
    cat = bn.nodes[1].cat        # A(out=j | in=i) = H[j][i]  (Table cat_hadamard)
    H = sim.mat_h()
    for (i, j), e in cat.items():
        assert np.isclose(e.value([], []), H[j, i])
    bn = C.circuit_to_bn(W.Circuit(n=2, ops=[("CNOT", 0, 1)], n_angles=0, noise=[]))
    cat = bn.nodes[2].cat        # Table cat_cnot
    assert set(cat) == {(0, 0, 0), (0, 1, 1), (1, 0, 1), (1, 1, 0)}


def _wmc(cnf, bn, theta, noise, evidence_nodes, values):
    """Weighted model count of the CNF with evidence clamped (brute force)."""
    clauses = [list(c) for c in cnf.clauses]
    for nd, u in zip(evidence_nodes, values):
        clauses.append([cnf.indicator[(nd, int(u))]])
    n = cnf.n_vars
    total = 0j
    # enumerate models by DFS with unit checks (tiny formulas only)
    assign = {}

    def sat_possible():
        for c in clauses:
            ok = False
            undecided = False
            for l in c:
                v = abs(l)
                if v not in assign:
                    undecided = True
                    continue
                if assign[v] == (l > 0):
                    ok = True
                    break
            if not ok and not undecided:
                return False
        return True

    def rec(v):
        nonlocal total
        if not sat_possible():
            return
        if v > n:
            w = 1 + 0j
            for wv, s in cnf.weight_var.items():
                if assign[wv]:
                    w *= s.value(theta, noise)
            total += w
            return
        for b in (False, True):
            assign[v] = b
            rec(v + 1)
            del assign[v]
    rec(1)
    return total


def test_cnf_weighted_model_count_is_branch_amplitude():
    # Sec. 3.2.1: models of the CNF are Feynman paths; their weighted count is
    # the amplitude.  Noisy Bell example (Table bn_to_cnf).
    circ = W.noisy_bell(0.36)
    bn = C.circuit_to_bn(circ)
    cnf = C.to_cnf(bn)
    assert cnf.dimacs().startswith("p cnf")
    ev_nodes = list(bn.outputs) + list(bn.events)
    for vals in itertools.product(range(2), range(2), range(2)):
        got = _wmc(cnf, bn, [], circ.noise, ev_nodes, vals)
        assert abs(got - oracle_amp(circ, [], list(vals))) < 1e-14


# ------------------------------------------------------------------ AC

@pytest.mark.parametrize("selectors", [True, False])
@pytest.mark.parametrize("name", sorted(CIRCUITS))
def test_ac_matches_oracle_on_every_assignment(name, selectors):
    circ = CIRCUITS[name]()
    ac = C.compile_circuit(circ, selectors=selectors)
    rng = np.random.default_rng(3)
    theta = rng.uniform(0, 2 * np.pi, size=circ.n_angles)
    for vals in all_assignments(circ):
        got = H.evaluate_assignment(ac, theta, vals)
        assert abs(got - oracle_amp(circ, theta, vals)) < 1e-13, vals


@pytest.mark.parametrize("selectors", [True, False])
@pytest.mark.parametrize("name", ["bell", "tiny", "ring3_dep"])
def test_ac_polynomial_identity_random_indicators(name, selectors):
    # Smooth and multilinear: AC(lambda) = sum_s f(s) prod_v lambda_{v, s_v}
    circ = CIRCUITS[name]()
    ac = C.compile_circuit(circ, selectors=selectors)
    rng = np.random.default_rng(5)
    theta = rng.uniform(0, 2 * np.pi, size=circ.n_angles)
    doms = circ.var_domains()
    lam = [rng.normal(size=d) + 1j * rng.normal(size=d) for d in doms]
    if math.prod(doms) > 20000:
        pytest.skip("state space too large for brute force")
    states = list(itertools.product(*[range(d) for d in doms]))
    expect = 0j
    for s in states:
        w = np.prod([lam[v][u] for v, u in enumerate(s)])
        expect += w * oracle_amp(circ, theta, list(s))
    got = H.evaluate(ac, theta, lam)
    assert abs(got - expect) < 1e-12 * max(1.0, abs(expect))


def test_ac_structure_invariants():
    for i in (1, 2, 4):
        ac = C.compile_circuit(W.config(i, small=True)["circuit"])
        lv = np.zeros(ac.n_internal, dtype=int)
        for l in range(ac.n_levels):
            lv[ac.level_ptr[l]:ac.level_ptr[l + 1]] = l
        assert ac.root == ac.n_internal - 1 and ac.level_ptr[-2] == ac.n_internal - 1
        for n in range(ac.n_internal):
            row = ac.col[ac.row_ptr[n]:ac.row_ptr[n + 1]]
            assert len(row) >= 1
            for r in row:
                if int(r) >> C.TAG_SHIFT == C.TAG_NODE:
                    assert lv[int(r) & ((1 << C.TAG_SHIFT) - 1)] < lv[n]


def test_qaoa_n32_p1_ac_is_paper_sized():
    # Table variational_problem_size_metrics lists 3139 nodes / 7959 edges for
    # the paper's compiler on this shape; ours must be of the same order.
    ac = C.compile_circuit(W.config(4, small=True)["circuit"])
    assert 500 < ac.n_internal < 20000 and ac.n_edges < 60000


def test_order_search_shrinks_ac_and_keeps_values():
    # The multi-start order may only lower the summed clique size of the
    # plain greedy run, and the AC it yields is the same polynomial.
    circ = W.qaoa_maxcut(8, W.random_regular_graph(8, 3, 11), 2, dep=0.004)
    one = C.compile_circuit(circ, order_trials=1)
    many = C.compile_circuit(circ, order_trials=64)
    assert many.n_internal <= one.n_internal
    rng = np.random.default_rng(2)
    theta = rng.uniform(0, 2 * np.pi, size=circ.n_angles)
    doms = circ.var_domains()
    for _ in range(20):
        vals = [0] * len(doms)
        vals[:circ.n] = [int(b) for b in rng.integers(0, 2, size=circ.n)]
        for v in rng.choice(np.arange(circ.n, len(doms)), size=3, replace=False):
            vals[int(v)] = int(rng.integers(0, doms[int(v)]))
        a = H.evaluate_assignment(many, theta, vals)
        b = oracle_amp(circ, theta, vals)
        assert abs(a - b) < 1e-13
        assert abs(H.evaluate_assignment(one, theta, vals) - b) < 1e-13


def test_c4_spot_amplitudes_match_path_sum():
    from oracle import pathsum
    n = 20
    edges = W.random_regular_graph(n, 3, 17)
    circ = W.qaoa_maxcut(n, edges, 1)
    ac = C.compile_circuit(circ)
    rng = np.random.default_rng(9)
    for _ in range(3):
        x = int(rng.integers(0, 1 << n))
        g, b = rng.uniform(0, 2 * np.pi, size=2)
        expect = pathsum.qaoa_p1_amplitude(n, edges, x, [g], [b])[0]
        got = H.evaluate_assignment(ac, [g, b], list(W.x_bits(x, n)))
        assert abs(got - expect) < 1e-13


# ------------------------------------------------------------------ blob

def test_blob_header_and_layout():
    circ = W.config(2, small=True)["circuit"]
    ac = C.compile_circuit(circ)
    b = blobmod.to_blob(ac)
    h = blobmod.blob_summary(b)
    assert h["magic"] == blobmod.MAGIC and h["version"] == 2
    assert h["n_selectors"] == len(ac.selectors) > 0
    assert h["n_int"] == ac.n_internal and h["n_edges"] == ac.n_edges
    assert h["n_vars"] == circ.n_vars and h["n_words"] == circ.n_words
    offs, widths, W_ = circ.var_layout()
    assert ac.var_offset == offs and ac.n_words == W_
    assert len(b) % 8 == 0


@pytest.mark.parametrize("seed", range(12))
def test_random_circuits_match_oracle(seed):
    # every op kind, CNOTs in both directions, negative and non-unit angle
    # scales, channels anywhere: the compiled AC against the branch state
    circ = W.random_circuit(seed)
    ac = C.compile_circuit(circ)
    rng = np.random.default_rng(seed)
    theta = rng.uniform(0, 2 * np.pi, size=circ.n_angles)
    states = list(all_assignments(circ))
    for i in rng.choice(len(states), size=min(120, len(states)), replace=False):
        vals = list(states[i])
        assert abs(H.evaluate_assignment(ac, theta, vals) - oracle_amp(circ, theta, vals)) < 1e-13, vals


def test_blob_cache_returns_the_same_blob(tmp_path):
    from paper_2103_17226_amd.blob import compile_blob, compile_blob_cached
    circ = W.config(2, small=True)["circuit"]
    b1, hit1 = compile_blob_cached(circ, str(tmp_path))
    b2, hit2 = compile_blob_cached(circ, str(tmp_path))
    assert (hit1, hit2) == (False, True) and b1 == b2 == compile_blob(circ)
    other = W.qaoa_maxcut(8, W.random_regular_graph(8, 3, 5), 1, dep=0.02)
    b3, hit3 = compile_blob_cached(other, str(tmp_path))
    assert not hit3 and b3 != b1
    assert compile_blob_cached(circ, "")[1] is False
