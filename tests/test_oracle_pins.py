"""Pins of the oracle against the paper's printed values, closed forms,
invariants and brute force -- never against itself.

Each test names what fixes the expected value.  ``test_oracle_mutations``
plants plausible mistakes in the oracle and shows that these pins catch them.
"""
import json
import os

import itertools

import numpy as np
import pytest

import workloads as W
from oracle import gibbs, grad, pathsum, sim, stats

GOLD = os.path.join(os.path.dirname(__file__), "golden")
SQ2 = np.sqrt(2.0)


def load_gold(name):
    with open(os.path.join(GOLD, name)) as f:
        return json.load(f)


# ---------------------------------------------------------------- closed forms

def test_gate_unitarity_and_kraus_completeness():
    for a in (0.0, 0.3, 2.1, -4.0):
        for U in (sim.mat_h(), sim.mat_rx(a), sim.mat_rz(a), sim.mat_x(), sim.mat_y(), sim.mat_z()):
            assert np.allclose(U.conj().T @ U, np.eye(2), atol=1e-15)
    for kind in ("DEP", "AD", "PD"):
        for p in (0.0, 0.01, 0.36, 1.0):
            s = sum(E.conj().T @ E for E in sim.kraus(kind, p))
            assert np.allclose(s, np.eye(2), atol=1e-15)


def test_hadamard_eq_q0m1():
    # Sec. 2.1, eq. q0m1: H|0> = (|0> + |1>)/sqrt(2)
    c = W.Circuit(n=1, ops=[("H", 0)], n_angles=0, noise=[])
    assert np.allclose(sim.statevector(c, []), [1 / SQ2, 1 / SQ2], atol=1e-16)


@pytest.mark.parametrize("a", [0.0, 0.4, 1.7, 3.3, 5.9])
def test_rotation_closed_forms(a):
    cx = W.Circuit(n=1, ops=[("RX", 0, 0, 1.0)], n_angles=1, noise=[])
    assert np.allclose(sim.statevector(cx, [a]), [np.cos(a / 2), -1j * np.sin(a / 2)], atol=1e-15)
    # RZ after H: relative phase e^{ia} between |1> and |0>
    cz = W.Circuit(n=1, ops=[("H", 0), ("RZ", 0, 0, 1.0)], n_angles=1, noise=[])
    psi = sim.statevector(cz, [a])
    assert np.allclose(psi, [np.exp(-0.5j * a) / SQ2, np.exp(0.5j * a) / SQ2], atol=1e-15)


def test_bit_order_and_cnot_truth_table():
    # X-like preparation on q0 only -> basis index 1 (LSB = q0)
    c = W.Circuit(n=3, ops=[("RX", 0, 0, 1.0)], n_angles=1, noise=[])
    psi = sim.statevector(c, [np.pi])
    assert np.isclose(abs(psi[1]), 1.0) and np.isclose(np.sum(abs(psi) ** 2), 1.0)
    # Table cat_cnot: control q0, target q1, all four inputs
    for x0 in (0, 1):
        for x1 in (0, 1):
            ops = []
            if x0:
                ops.append(("RX", 0, 0, 1.0))
            if x1:
                ops.append(("RX", 1, 0, 1.0))
            ops.append(("CNOT", 0, 1))
            psi = sim.statevector(W.Circuit(n=2, ops=ops, n_angles=1, noise=[]), [np.pi])
            out = x0 + 2 * (x1 ^ x0)
            assert np.isclose(abs(psi[out]), 1.0)


@pytest.mark.parametrize("n", [2, 3, 5, 8])
def test_bell_and_ghz(n):
    ops = [("H", 0)] + [("CNOT", q, q + 1) for q in range(n - 1)]
    psi = sim.statevector(W.Circuit(n=n, ops=ops, n_angles=0, noise=[]), [])
    expect = np.zeros(1 << n, dtype=complex)
    expect[0] = expect[-1] = 1 / SQ2
    assert np.allclose(psi, expect, atol=1e-15)


# ------------------------------------------------------------ worked example

def test_noisy_bell_worked_example():
    g = load_gold("noisy_bell.json")
    c = W.noisy_bell(g["gamma"])
    # rho after H, eq. density_matrix
    rh = sim.density_matrix(W.Circuit(n=1, ops=[("H", 0)], n_angles=0, noise=[]), [])
    assert np.allclose(rh, g["rho_after_h"], atol=1e-15)
    # rho after phase damping on the single qubit (Sec. 2.2.2)
    rp = sim.density_matrix(W.Circuit(n=1, ops=[("H", 0), ("PD", 0, 0)], n_angles=0,
                                      noise=[g["gamma"]]), [])
    assert np.allclose(rp, g["rho_after_pd"], atol=1e-15)
    # Table inference: branch amplitudes; |.| exact, sign per documented reading
    for rv in (0, 1):
        psi = sim.branch_state(c, [], [rv]) * SQ2
        ref = np.array(g["branch_amplitudes_times_sqrt2"][f"rv{rv}"])
        assert np.allclose(np.abs(psi), np.abs(ref), atol=1e-15)
        assert np.allclose(psi.imag, 0, atol=1e-15)
        bd = np.outer(psi, psi.conj()) / 2
        assert np.allclose(bd, g["branch_density_matrices"][f"rv{rv}"], atol=1e-15)
    # the oracle's reading: +sqrt(gamma) (Kraus form), the table's -0.6 differs by sign only
    a = sim.amplitude(c, [], 3, [1])
    assert np.isclose(a, -g["root_value_rv1_q0_1_q1_1"], atol=1e-15)
    # eq. final: the two components sum to the final density matrix
    assert np.allclose(sim.density_matrix(c, []), g["rho_final"], atol=1e-15)
    assert np.allclose(sim.probabilities_from_branches(c, []), np.diag(g["rho_final"]), atol=1e-15)
    # Table cat_phase_damping magnitudes are the Kraus entries
    E0, E1 = sim.kraus("PD", g["gamma"])
    assert np.isclose(E0[1, 1], g["pd_cat"]["q_in_1"][0]) and np.isclose(abs(E1[1, 1]), 0.6)


# ---------------------------------------------------------------- invariants

def _small_noisy(seed=3, dep=0.05, ad=None, n=4, p=1, ring=True):
    edges = W.ring_graph(n) if ring else W.random_regular_graph(n, 3, seed)
    return W.qaoa_maxcut(n, edges, p, dep=dep, ad=ad)


def test_dm_equals_sum_of_branch_outer_products():
    c = W.Circuit(n=2, ops=[("H", 0), ("DEP", 0, 0), ("CNOT", 0, 1), ("AD", 1, 1),
                            ("RX", 1, 0, 2.0), ("DEP", 1, 0)], n_angles=1, noise=[0.2, 0.3])
    th = [0.77]
    rho = sim.density_matrix(c, th)
    acc = np.zeros_like(rho)
    total = 0.0
    for k in sim.all_kraus_assignments(c):
        psi = sim.branch_state(c, th, k)
        acc += np.outer(psi, psi.conj())
        total += np.sum(np.abs(psi) ** 2)
    assert np.allclose(acc, rho, atol=1e-14)
    assert np.isclose(total, 1.0, atol=1e-14)      # Kraus completeness -> unit trace
    assert np.isclose(np.trace(rho).real, 1.0, atol=1e-14)


def test_unit_trace_qaoa_noisy():
    c = _small_noisy(dep=0.02, ad=0.01, n=4)
    for th in W.uniform_angles(3, 2, 11):
        assert np.isclose(np.trace(sim.density_matrix(c, th)).real, 1.0, atol=1e-13)


def test_gamma_zero_gives_uniform_even_with_depolarizing():
    c = W.qaoa_maxcut(6, W.random_regular_graph(6, 3, 1), 1, dep=0.03)
    for b in (0.3, 1.1, 2.9):
        p = sim.probabilities(c, [0.0, b])
        assert np.allclose(p, 1 / 64, atol=1e-14)


def test_bitflip_symmetry_and_ad_breaks_it():
    edges = W.random_regular_graph(6, 3, 2)
    th = [0.9, 0.4]
    idx = np.arange(64)
    for c in (W.qaoa_maxcut(6, edges, 1), W.qaoa_maxcut(6, edges, 1, dep=0.02)):
        p = sim.probabilities(c, th)
        assert np.allclose(p, p[idx ^ 63], atol=1e-14)
    p = sim.probabilities(W.qaoa_maxcut(6, edges, 1, dep=0.02, ad=0.05), th)
    assert np.max(np.abs(p - p[idx ^ 63])) > 1e-4


def test_amplitude_damping_relaxes_toward_the_ground_state():
    """Amplitude damping is the T1 (energy-relaxation) channel of Sec. 2.2,
    Table *noise models*: the excited state |1> decays to |0> with
    probability gamma and |0> is left alone.  Closed forms from the Kraus
    pair, checked through the density matrix and through the Kraus
    branches: AD(g)|1> gives P(0) = g; AD(g)|+> gives rho_00 = (1 + g)/2 and
    |rho_01| = sqrt(1 - g)/2; m rounds leave P(1) = (1 - g)^m."""
    g = 0.37
    one = W.Circuit(n=1, ops=[("RX", 0, 0, 1.0), ("AD", 0, 0)], n_angles=1, noise=[g])
    rho = sim.density_matrix(one, [np.pi])
    assert np.isclose(rho[0, 0].real, g, atol=1e-14)
    assert np.isclose(rho[1, 1].real, 1.0 - g, atol=1e-14)
    # branch amplitudes: k = 1 (the decay event) only lands on |0>
    f1 = sim.branch_state(one, [np.pi], k=[1])
    f0 = sim.branch_state(one, [np.pi], k=[0])
    assert np.isclose(abs(f1[0]) ** 2, g, atol=1e-14) and abs(f1[1]) < 1e-15
    assert np.isclose(abs(f0[1]) ** 2, 1.0 - g, atol=1e-14) and abs(f0[0]) < 1e-15
    zero = W.Circuit(n=1, ops=[("AD", 0, 0)], n_angles=0, noise=[g])
    assert np.allclose(sim.density_matrix(zero, []), [[1, 0], [0, 0]], atol=1e-15)
    plus = W.Circuit(n=1, ops=[("H", 0), ("AD", 0, 0)], n_angles=0, noise=[g])
    rho = sim.density_matrix(plus, [])
    assert np.isclose(rho[0, 0].real, (1.0 + g) / 2.0, atol=1e-14)
    assert np.isclose(abs(rho[0, 1]), np.sqrt(1.0 - g) / 2.0, atol=1e-14)
    m = 5
    rep = W.Circuit(n=1, ops=[("RX", 0, 0, 1.0)] + [("AD", 0, 0)] * m, n_angles=1, noise=[g])
    assert np.isclose(sim.probabilities(rep, [np.pi])[1], (1.0 - g) ** m, atol=1e-14)


def test_zero_noise_equivalence():
    edges = W.ring_graph(4)
    ideal = W.qaoa_maxcut(4, edges, 1)
    noisy = W.qaoa_maxcut(4, edges, 1, dep=0.0, ad=0.0)
    th = [1.2, 0.3]
    psi0 = sim.statevector(ideal, th)
    assert np.allclose(sim.branch_state(noisy, th), psi0, atol=1e-15)
    rng = np.random.default_rng(0)
    C = len(noisy.channels())
    for _ in range(5):
        k = rng.integers(0, 2, size=C)
        if k.sum() == 0:
            continue
        assert np.allclose(sim.branch_state(noisy, th, k), 0, atol=1e-15)


# ---------------------------------------------------------------- path sums

@pytest.mark.parametrize("n,seed", [(4, None), (6, 1), (8, 2), (10, 3), (12, 4)])
def test_pathsum_matches_statevector(n, seed):
    edges = W.ring_graph(n) if seed is None else W.random_regular_graph(n, 3, seed)
    c = W.qaoa_maxcut(n, edges, 1)
    ths = W.uniform_angles(3, 2, 99)
    rng = np.random.default_rng(n)
    for x in rng.integers(0, 1 << n, size=3):
        hist = pathsum.path_histogram(n, edges, int(x))
        assert int(hist.sum()) == 1 << n
        f = pathsum.amplitudes_from_histogram(hist, n, len(edges), ths[:, 0], ths[:, 1])
        for t, th in enumerate(ths):
            assert abs(f[t] - sim.statevector(c, th)[x]) < 1e-14


def test_p_layer_light_cone_matches_the_full_state_vector():
    """<Z_i Z_j> of QAOA with p = 1, 2, 3 from the restricted light-cone
    circuit against the full state vector, for every edge of 3-regular graphs
    and rings (on 16 qubits the cones are strict subsets), and against the
    p = 1 light cone."""
    rng = np.random.default_rng(23)
    for n, p, seed in ((10, 1, 1), (10, 2, 2), (16, 2, 3), (16, 2, -1), (14, 3, -1)):
        edges = W.random_regular_graph(n, 3, seed) if seed >= 0 else W.ring_graph(n)
        circ = W.qaoa_maxcut(n, edges, p)
        th = rng.uniform(0, 2 * np.pi, size=2 * p)
        psi = sim.statevector(circ, th)
        for (a, b) in edges:
            full = sim.zz_expectation(psi, a, b, n)
            assert abs(sim.qaoa_zz_lightcone(edges, th, a, b) - full) <= 1e-12
            if p == 1:
                assert abs(sim.qaoa_p1_zz_lightcone(edges, th[0], th[1], a, b) - full) <= 1e-12


def test_ring_transfer_matrix_amplitude_matches_path_sum_and_state_vector():
    """The ring transfer-matrix form against the brute-force path histogram
    (n <= 12) and the state vector (n <= 10); and its gamma = 0 closed form
    (a product state: |f|^2 = 2^-n) at n = 64."""
    rng = np.random.default_rng(17)
    for n in (3, 4, 7, 10, 12):
        edges = W.ring_graph(n)
        circ = W.qaoa_maxcut(n, edges, 1)
        g, b = rng.uniform(0, 2 * np.pi, size=2)
        psi = sim.statevector(circ, np.array([g, b])) if n <= 10 else None
        for x in rng.integers(0, 1 << n, size=4):
            f = pathsum.ring_amplitude(n, int(x), g, b)
            ref = pathsum.qaoa_p1_amplitude(n, edges, int(x), [g], [b])[0]
            assert abs(f - ref) <= 1e-13
            if psi is not None:
                assert abs(f - psi[int(x)]) <= 1e-13
    for x in (0, (1 << 64) - 1, 0x5A5A5A5A5A5A5A5A):
        f = pathsum.ring_amplitude(64, x, 0.0, 0.3)
        assert abs(abs(f) ** 2 - 2.0 ** -64) <= 1e-30


def test_pathsum_closed_forms_large_n():
    n = 24
    edges = W.random_regular_graph(n, 3, 5)
    x = 0xABCDE1
    hist = pathsum.path_histogram(n, edges, x)
    # beta = 0: |f|^2 = 2^-n for every x; gamma = 0: f = 2^{-n/2} e^{-i n beta}
    f = pathsum.amplitudes_from_histogram(hist, n, len(edges), [0.7, 0.0], [0.0, 0.45])
    assert np.isclose(abs(f[0]) ** 2, 2.0 ** -n, rtol=1e-12)
    assert abs(f[1] - 2.0 ** (-n / 2) * np.exp(-1j * n * 0.45)) < 1e-15


# ---------------------------------------------------------------- gradients

def test_product_rule_matches_finite_difference():
    c = _small_noisy(dep=0.03, ad=0.02, n=4, p=2)
    th = np.array([0.3, 1.1, 2.2, 0.6])
    rng = np.random.default_rng(1)
    k = np.zeros(len(c.channels()), dtype=int)
    k[rng.integers(0, len(k), size=3)] = 1
    g = grad.amplitude_grad(c, th, k)
    fd = grad.central_difference(lambda t: sim.branch_state(c, t, k), th, h=1e-6)
    assert np.allclose(g, fd, atol=1e-8)


def _tiny_angle_circuit():
    ops = [("H", 0), ("H", 1), ("CNOT", 0, 1), ("DEP", 1, 0), ("RZ", 1, 0, 2.0), ("AD", 0, 1),
           ("CNOT", 0, 1), ("RX", 0, 1, 2.0), ("RX", 1, 1, 2.0), ("DEP", 0, 0),
           ("RZ", 0, 2, 2.0), ("RX", 1, 3, 2.0)]
    return W.Circuit(n=2, ops=ops, n_angles=4, noise=[0.07, 0.2], edges=[(0, 1)])


def test_param_shift_matches_fd():
    c = _small_noisy(dep=0.02, ad=0.01, n=3, p=2, ring=True)
    th = np.array([0.8, 0.25, 1.9, 2.7])
    ps = grad.expected_cost_param_shift(c, th)
    fd = grad.central_difference(lambda t: sim.expected_cost(c, t), th, h=1e-5)
    assert np.allclose(ps, fd, atol=1e-8)


def test_param_shift_matches_product_rule_through_branches():
    c = _tiny_angle_circuit()
    th = np.array([0.8, 0.25, 1.9, 2.7])
    ps = grad.expected_cost_param_shift(c, th)
    # d<C>/dtheta = sum_k sum_x C(x) 2 Re(conj f df) (product rule per branch)
    C = sim.cost_vector(c)
    acc = np.zeros(4)
    for k in sim.all_kraus_assignments(c):
        f = sim.branch_state(c, th, k)
        df = grad.amplitude_grad(c, th, k)
        acc += 2 * np.real(np.conj(f)[None, :] * df) @ C
    assert np.allclose(acc, ps, atol=1e-12)
    assert np.max(np.abs(ps)) > 1e-3


# ---------------------------------------------------------------- Gibbs / RNG

def test_splitmix64_reference_values():
    # SplitMix64 seeded with state 0 (Steele, Lea, Flood 2014): the first two
    # outputs of the published generator.
    assert gibbs.mix64(0) == 0xE220A8397B1DCDAF
    assert gibbs.mix64(gibbs.GOLDEN) == 0x6E789E6AA1B965F4
    u = [gibbs.uniform(7, c, s, v) for c in range(4) for s in range(4) for v in range(4)]
    assert all(0.0 <= x < 1.0 for x in u) and len(set(u)) == len(u)


def test_choose_rule():
    assert gibbs.choose([0.0, 0.0], 0.3) is None
    assert gibbs.choose([1.0, 1.0], 0.0) == 0
    assert gibbs.choose([1.0, 1.0], 0.5) == 1          # strict '<': 1.0 < 1.0 false
    assert gibbs.choose([0.0, 2.0, 0.0], 0.999999) == 1
    assert gibbs.choose([1.0, 0.0, 3.0], 0.26) == 2


def test_exact_kernel_is_stationary():
    c = W.noisy_bell(0.36)
    states, d0 = gibbs.exact_sweep_distribution(c, [], 0)
    pi = np.array([abs(gibbs.BranchCache(c, []).amp(s)) ** 2 for s in states.tolist()])
    # run the exact kernel from pi itself: must stay at pi
    _, d1 = gibbs.exact_sweep_distribution(c, [], 1)
    _, d50 = gibbs.exact_sweep_distribution(c, [], 50)
    assert np.isclose(pi.sum(), 1.0)
    # the noisy Bell chain converges to |f|^2 within 50 sweeps
    assert np.allclose(d50, pi, atol=1e-10)
    assert np.isclose(d1.sum(), 1.0)


def test_reference_chain_matches_exact_sweep_distribution():
    edges = W.ring_graph(3)
    c = W.qaoa_maxcut(3, edges, 1)
    th = [0.6, 0.35]
    t = 2
    states, dist = gibbs.exact_sweep_distribution(c, th, t)
    counts = np.zeros(len(states))
    index = {tuple(s): i for i, s in enumerate(states.tolist())}
    for ch in range(3000):
        samp, _ = gibbs.run_chain(c, th, seed=5, chain=ch, burn_in=t - 1, thin=1, n_samples=1)
        counts[index[tuple(samp[0])]] += 1
    _, _, pval = stats.chi2_pooled(counts, dist)
    assert pval > 1e-3


def test_resumed_reference_chain_is_the_same_chain():
    # Resuming from the final state with the sweep count continues the chain;
    # a wrong sweep number changes the random stream and the samples.
    c = W.qaoa_maxcut(3, W.ring_graph(3), 1, dep=0.05, ad=0.03)
    th = [0.9, 0.3]
    for ch in range(5):
        whole, _ = gibbs.run_chain(c, th, seed=8, chain=ch, burn_in=2, thin=1, n_samples=6)
        part, last = gibbs.run_chain(c, th, seed=8, chain=ch, burn_in=2, thin=1, n_samples=3)
        rest, _ = gibbs.run_chain(c, th, seed=8, chain=ch, burn_in=0, thin=1, n_samples=3, init=last,
                                  first_sweep=5)
        assert np.array_equal(np.concatenate([part, rest]), whole)
    # the exact kernel from a point mass: the resumed reference chain from
    # state s has the law of one sweep from s (chi-square over many chains)
    c = W.Circuit(n=2, ops=[("H", 0), ("DEP", 0, 0), ("H", 1), ("CNOT", 0, 1), ("AD", 1, 1),
                            ("RX", 0, 1, 2.0), ("RZ", 1, 0, 2.0)],
                  n_angles=2, noise=[0.3, 0.25], edges=[(0, 1)])
    s0 = [1, 0, 2, 1]
    counts = {}
    for ch in range(2000):
        smp, _ = gibbs.run_chain(c, th, seed=3, chain=ch, burn_in=0, thin=1, n_samples=1, init=s0,
                                 first_sweep=11)
        counts[tuple(smp[0])] = counts.get(tuple(smp[0]), 0) + 1
    law = _one_sweep_law(c, th, s0)
    keys = sorted(law)
    obs = np.array([counts.get(k, 0) for k in keys])
    assert sum(counts.get(k, 0) for k in counts if k not in law) == 0
    _, _, pval = stats.chi2_pooled(obs, np.array([law[k] for k in keys]))
    assert pval > 1e-3


def _one_sweep_law(c, th, s0):
    """Law of one systematic sweep from s0, by enumerating every branch of the
    single-site updates (each update draws u with |f(s[v<-u])|^2 / sum)."""
    bc = gibbs.BranchCache(c, th)
    doms = c.var_domains()
    law = {tuple(s0): 1.0}
    for v in range(c.n_vars):
        nxt = {}
        for s, p in law.items():
            w = []
            for u in range(doms[v]):
                t = list(s)
                t[v] = u
                w.append(abs(bc.amp(t)) ** 2)
            tot = sum(w)
            if tot == 0:
                nxt[s] = nxt.get(s, 0) + p
                continue
            for u in range(doms[v]):
                if w[u] > 0:
                    t = list(s)
                    t[v] = u
                    nxt[tuple(t)] = nxt.get(tuple(t), 0) + p * w[u] / tot
        law = nxt
    return law


def test_lightcone_zz_equals_full_state_vector():
    # p = 1 QAOA: the light-cone value of <Z_i Z_j> equals the full state
    # vector's on every edge and on non-edges (n = 10, 3-regular).
    edges = W.random_regular_graph(10, 3, 21)
    circ = W.qaoa_maxcut(10, edges, 1)
    rng = np.random.default_rng(6)
    for _ in range(3):
        g, b = rng.uniform(0, 2 * np.pi, size=2)
        psi = sim.statevector(circ, [g, b])
        for (i, j) in list(edges) + [(0, 5), (2, 9)]:
            full = sim.zz_expectation(psi, i, j, 10)
            assert abs(sim.qaoa_p1_zz_lightcone(edges, g, b, i, j) - full) < 1e-12
    # closed form at gamma = 0 (no entanglement): <ZZ> = 0
    assert abs(sim.qaoa_p1_zz_lightcone(edges, 0.0, 0.7, *edges[0])) < 1e-12


def test_vqe_ising_single_site_closed_form():
    # one site: H, RZ(2 h beta), RX(2 alpha) |0> gives P(1) = (1 - sin 2alpha sin 2h beta) / 2
    rng = np.random.default_rng(13)
    for hval in (1.0, -1.0):
        circ = W.vqe_ising(1, 1, 1, [], [hval])
        for _ in range(4):
            g, b, a = rng.uniform(0, 2 * np.pi, size=3)
            psi = sim.statevector(circ, [g, b, a])
            want = (1 - np.sin(2 * a) * np.sin(2 * hval * b)) / 2
            assert abs(abs(psi[1]) ** 2 - want) < 1e-14


def test_vqe_ising_closed_forms_on_a_grid():
    edges, J, h = W.ising_instance(2, 3, 5)
    circ = W.vqe_ising(2, 3, 2, J, h, dep=0.02)
    n = circ.n
    # no coupling and no field phase: |+>^n is an X eigenstate, P(x) = 2^-n under depolarizing noise too
    for th in ([0.0, 0.0, 0.7, 0.0, 0.0, 1.9], [0.0, 0.0, 2.3, 0.0, 0.0, 0.4]):
        assert np.allclose(sim.probabilities(circ, th), 1.0 / 2 ** n, atol=1e-14)
    # the energy function: all spins up (x = 0) gives sum J + sum h
    assert W.ising_energy(edges, J, h, np.zeros((1, n), dtype=int))[0] == sum(J) + sum(h)
    bits = np.array([[1, 0, 1, 1, 0, 0]])
    s = 1 - 2 * bits[0]
    want = sum(Jij * s[i] * s[j] for (i, j), Jij in zip(edges, J)) + sum(hi * s[i] for i, hi in enumerate(h))
    assert W.ising_energy(edges, J, h, bits)[0] == want


def _tiny_noisy_for_posterior():
    return W.Circuit(n=2, ops=[("H", 0), ("DEP", 0, 0), ("H", 1), ("CNOT", 0, 1), ("AD", 1, 1),
                               ("RX", 0, 1, 2.0), ("RZ", 1, 0, 2.0), ("DEP", 1, 0)],
                     n_angles=2, noise=[0.3, 0.25], edges=[(0, 1)])


def test_conditional_reference_chain_targets_the_error_posterior():
    # with the outputs held (first_var = n), the chain's law converges to
    # P(k | x) proportional to |f(x, k)|^2 over the noise events
    circ = _tiny_noisy_for_posterior()
    th = [0.8, 1.3]
    x = [1, 0]
    doms = circ.var_domains()[circ.n:]
    ks = list(itertools.product(*[range(d) for d in doms]))
    post = np.array([abs(sim.amplitude(circ, th, x[0] + 2 * x[1], k)) ** 2 for k in ks])
    post /= post.sum()
    index = {k: i for i, k in enumerate(ks)}
    counts = np.zeros(len(ks))
    for ch in range(3000):
        smp, _ = gibbs.run_chain(circ, th, seed=31, chain=ch, burn_in=14, thin=1, n_samples=1,
                                 init=x + [0] * len(doms), first_var=circ.n)
        assert list(smp[0][:circ.n]) == x
        counts[index[tuple(smp[0][circ.n:])]] += 1
    _, _, pval = stats.chi2_pooled(counts, post)
    assert pval > 1e-3


def test_chi2_detects_bias_and_accepts_truth():
    rng = np.random.default_rng(0)
    p = rng.dirichlet(np.ones(20))
    good = np.bincount(rng.choice(20, size=20000, p=p), minlength=20)
    assert stats.chi2_pooled(good, p)[2] > 1e-3
    q = p.copy()
    q[0] *= 1.3
    q /= q.sum()
    bad = np.bincount(rng.choice(20, size=20000, p=q), minlength=20)
    assert stats.chi2_pooled(bad, p)[2] < 1e-3
    assert stats.kl_divergence(good, p) < stats.kl_divergence(bad, p)


def test_most_probable_events_closed_forms():
    # Sec. 5: the noise events that best explain an outcome, by the largest
    # joint probability P(x, k) = |f(x, k)|^2.  One depolarizing channel on
    # |0>: outcome 1 needs an X or a Y error, P = p/3 each (a tie); outcome 0
    # is best explained by no error, P = 1 - p.
    p = 0.12
    dep = W.Circuit(n=1, ops=[("DEP", 0, 0)], n_angles=0, noise=[p], edges=[])
    best, ks = sim.most_probable_events(dep, [], 1)
    assert best == pytest.approx(p / 3, rel=1e-14) and ks == [(1,), (2,)]
    best, ks = sim.most_probable_events(dep, [], 0)
    assert best == pytest.approx(1 - p, rel=1e-14) and ks == [(0,)]
    # |1> then amplitude damping: outcome 0 only through a decay (P = gamma)
    g = 0.3
    ad = W.Circuit(n=1, ops=[("RX", 0, 0, 1.0), ("AD", 0, 0)], n_angles=1, noise=[g], edges=[])
    best, ks = sim.most_probable_events(ad, [np.pi], 0)
    assert best == pytest.approx(g, rel=1e-12) and ks == [(1,)]
    best, ks = sim.most_probable_events(ad, [np.pi], 1)
    assert best == pytest.approx(1 - g, rel=1e-12) and ks == [(0,)]
    # both in a row: outcome 0 comes from a decay with no Pauli error
    # (gamma (1 - p)), or no decay and an X or Y error ((1 - gamma) p / 3)
    both = W.Circuit(n=1, ops=[("RX", 0, 0, 1.0), ("AD", 0, 0), ("DEP", 0, 1)], n_angles=1, noise=[0.3, 0.3],
                     edges=[])
    best, ks = sim.most_probable_events(both, [np.pi], 0)
    assert best == pytest.approx(0.3 * 0.7, rel=1e-12) and ks == [(1, 0)]
    both.noise = [0.05, 0.6]
    best, ks = sim.most_probable_events(both, [np.pi], 0)
    assert best == pytest.approx(0.95 * 0.2, rel=1e-12) and ks == [(0, 1), (0, 2)]
    # the best branch never exceeds the outcome's probability, the sum over k
    assert best <= sim.probabilities(both, [np.pi])[0] + 1e-15
