"""Plant plausible mistakes in the oracle (on the CPU) and check that the
pins in ``test_oracle_pins`` catch every one of them."""
import numpy as np
import pytest

import tests.test_oracle_pins as pins
from oracle import gibbs, grad, sim


def _fails(fn, *args):
    with pytest.raises(AssertionError):
        fn(*args)


def test_rx_sign_flip_is_caught(monkeypatch):
    good = sim.mat_rx
    monkeypatch.setattr(sim, "mat_rx", lambda a: good(a).conj())
    _fails(pins.test_rotation_closed_forms, 0.4)
    _fails(pins.test_pathsum_matches_statevector, 6, 1)


def test_rz_sign_flip_is_caught(monkeypatch):
    good = sim.mat_rz
    monkeypatch.setattr(sim, "mat_rz", lambda a: good(-a))
    _fails(pins.test_rotation_closed_forms, 0.4)
    _fails(pins.test_pathsum_matches_statevector, 8, 2)


def test_depolarizing_split_is_caught(monkeypatch):
    good = sim.kraus

    def bad(kind, p):
        ks = good(kind, p)
        if kind == "DEP":
            ks = [ks[0]] + [E * np.sqrt(3.0) for E in ks[1:]]   # p instead of p/3
        return ks
    monkeypatch.setattr(sim, "kraus", bad)
    _fails(pins.test_gate_unitarity_and_kraus_completeness)
    _fails(pins.test_unit_trace_qaoa_noisy)


def test_transposed_operand_is_caught(monkeypatch):
    good = sim.apply_1q
    monkeypatch.setattr(sim, "apply_1q", lambda psi, U, q, n: good(psi, U.T, q, n))
    _fails(pins.test_dm_equals_sum_of_branch_outer_products)


def test_swapped_cnot_is_caught(monkeypatch):
    good = sim.apply_cnot
    monkeypatch.setattr(sim, "apply_cnot", lambda psi, c, t, n: good(psi, t, c, n))
    _fails(pins.test_bit_order_and_cnot_truth_table)


def test_reversed_bit_order_is_caught(monkeypatch):
    good = sim.apply_1q
    monkeypatch.setattr(sim, "apply_1q", lambda psi, U, q, n: good(psi, U, n - 1 - q, n))
    _fails(pins.test_bit_order_and_cnot_truth_table)


def test_dropped_kraus_term_is_caught(monkeypatch):
    good = sim.kraus
    monkeypatch.setattr(sim, "kraus", lambda kind, p: good(kind, p)[:-1])
    _fails(pins.test_unit_trace_qaoa_noisy)


def test_missing_chain_factor_is_caught(monkeypatch):
    monkeypatch.setattr(grad, "angle_gates",
                        lambda circ, j: [(i, 1.0) for i, op in enumerate(circ.ops)
                                         if op[0] in ("RZ", "RX") and op[2] == j])
    _fails(pins.test_param_shift_matches_fd)


def test_wrong_shift_is_caught(monkeypatch):
    good = sim.expected_cost

    def bad(circ, theta, noise=None, shift=None):
        if shift:
            shift = {k: v / 2 for k, v in shift.items()}
        return good(circ, theta, noise, shift)
    monkeypatch.setattr(sim, "expected_cost", bad)
    _fails(pins.test_param_shift_matches_fd)


def test_wrong_mixer_constant_is_caught(monkeypatch):
    monkeypatch.setattr(gibbs, "GOLDEN", 0x9E3779B97F4A7C13)
    _fails(pins.test_splitmix64_reference_values)


def test_amplitude_instead_of_probability_weights_is_caught(monkeypatch):
    def bad(bc, state, v):
        dom = bc.circ.var_domains()[v]
        out = []
        s = list(state)
        for u in range(dom):
            s[v] = u
            out.append(abs(bc.amp(s)))
        return out
    monkeypatch.setattr(gibbs, "conditional_weights", bad)
    _fails(pins.test_reference_chain_matches_exact_sweep_distribution)


def test_amplitude_damping_toward_the_excited_state_is_caught(monkeypatch):
    good = sim.kraus

    def bad(kind, p):
        if kind == "AD":            # the mirrored channel: decays |0> -> |1>
            return [np.array([[np.sqrt(1.0 - p), 0], [0, 1]], dtype=np.complex128),
                    np.array([[0, 0], [np.sqrt(p), 0]], dtype=np.complex128)]
        return good(kind, p)
    monkeypatch.setattr(sim, "kraus", bad)
    # still a complete channel that breaks bit-flip symmetry ...
    pins.test_gate_unitarity_and_kraus_completeness()
    pins.test_bitflip_symmetry_and_ad_breaks_it()
    # ... but not the relaxation to |0>
    _fails(pins.test_amplitude_damping_relaxes_toward_the_ground_state)
