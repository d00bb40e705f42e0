"""State-vector, Kraus-branch and density-matrix simulators (complex128).

Test infrastructure only (see ``oracle/__init__.py``).

Conventions: amplitude index = sum_q x_q 2^q (qubit 0 is the least
significant bit).  The paper prints its two-qubit vectors with q0 as the left
tensor factor (Sec. 2.1); that is a display order only and every printed
result used here is invariant under it.
"""
from __future__ import annotations

import numpy as np

# ---------------------------------------------------------------------------
# gate and Kraus matrices
# ---------------------------------------------------------------------------

SQ2 = 1.0 / np.sqrt(2.0)


def mat_h():
    """Hadamard, Sec. 2.1 (the unitary printed there)."""
    return np.array([[SQ2, SQ2], [SQ2, -SQ2]], dtype=np.complex128)


def mat_x():
    return np.array([[0, 1], [1, 0]], dtype=np.complex128)


def mat_y():
    return np.array([[0, -1j], [1j, 0]], dtype=np.complex128)


def mat_z():
    return np.array([[1, 0], [0, -1]], dtype=np.complex128)


def mat_rz(a):
    """RZ(a) = exp(-i a Z / 2)."""
    return np.array([[np.exp(-0.5j * a), 0], [0, np.exp(0.5j * a)]], dtype=np.complex128)


def mat_rx(a):
    """RX(a) = exp(-i a X / 2)."""
    c, s = np.cos(0.5 * a), np.sin(0.5 * a)
    return np.array([[c, -1j * s], [-1j * s, c]], dtype=np.complex128)


def dmat_rz(a):
    """d RZ(a) / d a."""
    return np.array([[-0.5j * np.exp(-0.5j * a), 0], [0, 0.5j * np.exp(0.5j * a)]],
                    dtype=np.complex128)


def dmat_rx(a):
    """d RX(a) / d a."""
    c, s = np.cos(0.5 * a), np.sin(0.5 * a)
    return np.array([[-0.5 * s, -0.5j * c], [-0.5j * c, -0.5 * s]], dtype=np.complex128)


def kraus(kind, prob):
    """Kraus operators of the canonical channels (Sec. 2.2, Table
    "noise models"; the phase-damping pair is the one printed in Sec. 2.2.2).

    DEP: symmetric depolarizing with *total* error probability prob, split
         evenly over X, Y, Z (the evaluation's "probability that one of
         Pauli-X, Y, or Z noise events may happen").
    AD:  amplitude damping with decay probability prob.
    PD:  phase damping with parameter prob.
    """
    if kind == "DEP":
        a = np.sqrt(1.0 - prob)
        b = np.sqrt(prob / 3.0)
        return [a * np.eye(2, dtype=np.complex128), b * mat_x(), b * mat_y(), b * mat_z()]
    if kind == "AD":
        return [np.array([[1, 0], [0, np.sqrt(1.0 - prob)]], dtype=np.complex128),
                np.array([[0, np.sqrt(prob)], [0, 0]], dtype=np.complex128)]
    if kind == "PD":
        return [np.array([[1, 0], [0, np.sqrt(1.0 - prob)]], dtype=np.complex128),
                np.array([[0, 0], [0, np.sqrt(prob)]], dtype=np.complex128)]
    raise ValueError(kind)


CHANNELS = ("DEP", "AD", "PD")


def gate_matrix(op, theta, shift=0.0):
    """2x2 matrix of a single-qubit gate op; shift is added to its angle."""
    name = op[0]
    if name == "H":
        return mat_h()
    if name == "RZ":
        return mat_rz(op[3] * theta[op[2]] + shift)
    if name == "RX":
        return mat_rx(op[3] * theta[op[2]] + shift)
    raise ValueError(name)


# ---------------------------------------------------------------------------
# primitive actions on a 2^n vector
# ---------------------------------------------------------------------------

def apply_1q(psi, U, q, n):
    """psi' = (I x .. U on qubit q .. x I) psi."""
    t = psi.reshape(1 << (n - q - 1), 2, 1 << q)
    out = np.einsum("ab,ibj->iaj", U, t)
    return out.reshape(-1)


def apply_cnot(psi, c, t, n):
    """CNOT: target bit t flipped where control bit c is 1."""
    idx = np.arange(1 << n)
    src = np.where((idx >> c) & 1, idx ^ (1 << t), idx)
    return psi[src]


def zero_state(n):
    psi = np.zeros(1 << n, dtype=np.complex128)
    psi[0] = 1.0
    return psi


# ---------------------------------------------------------------------------
# pure states: ideal circuits and single Kraus branches
# ---------------------------------------------------------------------------

def branch_state(circ, theta, k=None, noise=None, override=None):
    """O_M ... O_1 |0^n>, where each gate is its unitary and each channel c is
    its *unnormalized* Kraus operator E_{k[c]} (Sec. 3.1, noise events as
    random variables whose table holds the Kraus amplitudes).

    k: Kraus index per channel, in circuit order (None: all zeros).
    override: optional {op_index: 2x2 matrix} replacing a gate's matrix
    (used by the product-rule derivative).
    """
    theta = np.asarray(theta, dtype=np.float64)
    noise = circ.noise if noise is None else noise
    n = circ.n
    psi = zero_state(n)
    c = 0
    for i, op in enumerate(circ.ops):
        name = op[0]
        if name in CHANNELS:
            kc = 0 if k is None else int(k[c])
            psi = apply_1q(psi, kraus(name, noise[op[2]])[kc], op[1], n)
            c += 1
        elif name == "CNOT":
            psi = apply_cnot(psi, op[1], op[2], n)
        else:
            U = override[i] if (override and i in override) else gate_matrix(op, theta)
            psi = apply_1q(psi, U, op[1], n)
    return psi


def statevector(circ, theta):
    """Ideal state vector U(theta)|0^n>; refuses circuits with channels."""
    if any(op[0] in CHANNELS for op in circ.ops):
        raise ValueError("circuit has noise channels; use branch_state or density_matrix")
    return branch_state(circ, theta)


def amplitude(circ, theta, x_index, k=None, noise=None):
    """Branch amplitude f(x, k) = <x| O_M ... O_1 |0^n>."""
    return branch_state(circ, theta, k, noise)[int(x_index)]


def all_kraus_assignments(circ):
    """Every Kraus-index tuple k (only for tiny circuits)."""
    doms = [4 if op[0] == "DEP" else 2 for op in circ.ops if op[0] in CHANNELS]
    grids = np.meshgrid(*[np.arange(d) for d in doms], indexing="ij") if doms else []
    if not doms:
        return np.zeros((1, 0), dtype=np.int64)
    return np.stack([g.reshape(-1) for g in grids], axis=1)


# ---------------------------------------------------------------------------
# mixed states
# ---------------------------------------------------------------------------

def _apply_1q_rho(rho, U, q, n):
    d = 1 << n
    # rho -> U rho U^dagger on qubit q
    r = rho.reshape(1 << (n - q - 1), 2, 1 << q, d)
    r = np.einsum("ab,ibjk->iajk", U, r).reshape(d, d)
    r = r.reshape(d, 1 << (n - q - 1), 2, 1 << q)
    r = np.einsum("ab,kibj->kiaj", U.conj(), r).reshape(d, d)
    return r


def density_matrix(circ, theta, noise=None, shift=None):
    """rho <- U rho U^dagger for gates, rho <- sum_k E_k rho E_k^dagger for
    channels (Sec. 2.2.2), starting from |0^n><0^n|.

    shift: optional {op_index: angle offset} (parameter-shift rule).
    """
    theta = np.asarray(theta, dtype=np.float64)
    noise = circ.noise if noise is None else noise
    n = circ.n
    d = 1 << n
    rho = np.zeros((d, d), dtype=np.complex128)
    rho[0, 0] = 1.0
    idx = np.arange(d)
    for i, op in enumerate(circ.ops):
        name = op[0]
        if name in CHANNELS:
            acc = np.zeros_like(rho)
            for E in kraus(name, noise[op[2]]):
                acc += _apply_1q_rho(rho, E, op[1], n)
            rho = acc
        elif name == "CNOT":
            src = np.where((idx >> op[1]) & 1, idx ^ (1 << op[2]), idx)
            rho = rho[np.ix_(src, src)]
        else:
            s = 0.0 if not shift else shift.get(i, 0.0)
            rho = _apply_1q_rho(rho, gate_matrix(op, theta, s), op[1], n)
    return rho


def probabilities(circ, theta, noise=None, shift=None):
    """P(x) = rho_xx."""
    return np.real(np.diag(density_matrix(circ, theta, noise, shift))).copy()


def probabilities_from_branches(circ, theta, noise=None):
    """P(x) = sum_k |f(x,k)|^2 by enumerating every Kraus branch (tiny only)."""
    p = np.zeros(1 << circ.n)
    for k in all_kraus_assignments(circ):
        p += np.abs(branch_state(circ, theta, k, noise)) ** 2
    return p


def cost_vector(circ):
    """MaxCut cost C(x) = number of cut edges, for every basis index x."""
    idx = np.arange(1 << circ.n)
    c = np.zeros(1 << circ.n)
    for i, j in circ.edges:
        c += (((idx >> i) ^ (idx >> j)) & 1)
    return c


def expected_cost(circ, theta, noise=None, shift=None):
    return float(np.dot(probabilities(circ, theta, noise, shift), cost_vector(circ)))


# ---------------------------------------------------------------------------
# local observables of large noise-free QAOA circuits
# ---------------------------------------------------------------------------

class _Ops:
    """Minimal circuit record (n, ops, noise) for the simulators above."""

    def __init__(self, n, ops):
        self.n, self.ops, self.noise = n, ops, []


def zz_expectation(psi, i, j, n):
    """<Z_i Z_j> of a state vector (qubit q = bit q of the index)."""
    idx = np.arange(1 << n)
    sign = 1.0 - 2.0 * (((idx >> i) ^ (idx >> j)) & 1)
    return float(np.dot(np.abs(psi) ** 2, sign))


def qaoa_p1_zz_lightcone(edges, gamma, beta, i, j):
    """<Z_i Z_j> after one QAOA layer (H on all, exp(-i gamma Z_a Z_b) per edge
    as CNOT-RZ(2 gamma)-CNOT, RX(2 beta) on all) from the reverse light cone.

    In U^dag Z_i Z_j U the mixers on qubits other than i, j commute with
    Z_i Z_j and cancel, and so do the phase gates of edges touching neither i
    nor j; what remains acts on i, j and their neighbours only, so the value
    is that of the same circuit on those qubits with the edges incident to
    i or j (textbook locality of p = 1 QAOA)."""
    inc = sorted({tuple(sorted(e)) for e in edges if i in e or j in e})
    cone = sorted({q for e in inc for q in e} | {i, j})
    pos = {q: k for k, q in enumerate(cone)}
    m = len(cone)
    ops = [("H", q) for q in range(m)]
    for a, b in inc:
        ops += [("CNOT", pos[a], pos[b]), ("RZ", pos[b], 0, 2.0), ("CNOT", pos[a], pos[b])]
    ops += [("RX", q, 1, 2.0) for q in range(m)]
    psi = branch_state(_Ops(m, ops), [gamma, beta])
    return zz_expectation(psi, pos[i], pos[j], m)


def qaoa_zz_lightcone(edges, theta, i, j):
    """<Z_i Z_j> after p QAOA layers (theta = [gamma_1, beta_1, ..., gamma_p,
    beta_p], the circuit of qaoa_p1_zz_lightcone repeated per layer) from the
    reverse light cone.

    Pulled back through the last layer, Z_i Z_j acts on i, j and their
    neighbours; through each earlier layer its support grows by one more ring
    of neighbours, so after p layers it lies in the qubits within graph
    distance p of {i, j}.  A gate on an edge with an endpoint farther away
    never meets the operator, and gates inside that set that do not meet it
    commute with it and cancel, so the value is that of the circuit restricted
    to that set with every edge inside it (textbook locality of QAOA)."""
    p = len(theta) // 2
    und = {tuple(sorted(e)) for e in edges}
    nbr = {}
    for a, b in und:
        nbr.setdefault(a, set()).add(b)
        nbr.setdefault(b, set()).add(a)
    cone = {i, j}
    for _ in range(p):
        cone |= {b for a in cone for b in nbr.get(a, ())}
    cone = sorted(cone)
    pos = {q: k for k, q in enumerate(cone)}
    inner = sorted(e for e in und if e[0] in pos and e[1] in pos)
    m = len(cone)
    ops = [("H", q) for q in range(m)]
    for layer in range(p):
        for a, b in inner:
            ops += [("CNOT", pos[a], pos[b]), ("RZ", pos[b], 2 * layer, 2.0), ("CNOT", pos[a], pos[b])]
        ops += [("RX", q, 2 * layer + 1, 2.0) for q in range(m)]
    psi = branch_state(_Ops(m, ops), list(theta))
    return zz_expectation(psi, pos[i], pos[j], m)


# ---------------------------------------------------------------------------
# most probable explanation of an outcome (Sec. 5)
# ---------------------------------------------------------------------------

def most_probable_events(circ, theta, x_index, noise=None, rtol=1e-12):
    """The noise events that best explain an observed outcome x: the joint
    probability of outcome and events is P(x, k) = |f(x, k)|^2 (a real error
    probability, where the maximum is defined, unlike for amplitudes), so
    k* = argmax_k |f(x, k)|^2 over every Kraus-index tuple (tiny circuits
    only).  Returns (max_k P(x, k), every k within rtol of the maximum, in
    enumeration order)."""
    ks = all_kraus_assignments(circ)
    p = np.array([abs(amplitude(circ, theta, x_index, k, noise)) ** 2 for k in ks])
    best = float(p.max())
    tie = np.nonzero(p >= best * (1.0 - rtol))[0]
    return best, [tuple(int(v) for v in ks[i]) for i in tie]
