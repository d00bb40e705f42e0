"""Exact derivatives for the oracle (complex128 / float64).

Test infrastructure only (see ``oracle/__init__.py``).

Gradients via model counting are among the queries the toolchain mirrors
(Sec. 5).  Three independent routes are provided so that each can check the
others:

* ``amplitude_grad``: the product rule.  f(x,k;theta) is a product of
  per-op matrices, so d f / d theta_j is the sum, over every gate whose angle
  is s * theta_j, of the same product with that gate's matrix replaced by
  s * dU/da.
* ``expected_cost_param_shift``: the parameter-shift rule for gates
  exp(-i a P / 2) with P a Pauli: d<C>/da = (<C>(a + pi/2) - <C>(a - pi/2)) / 2
  (a textbook identity, not from the paper), summed over every gate that uses
  theta_j with the chain factor s.
* ``central_difference``: symmetric finite differences of any function.
"""
from __future__ import annotations

import numpy as np

from . import sim


def angle_gates(circ, j):
    """Indices and scale factors of the gates whose angle is s * theta[j]."""
    return [(i, op[3]) for i, op in enumerate(circ.ops)
            if op[0] in ("RZ", "RX") and op[2] == j]


def amplitude_grad(circ, theta, k=None, noise=None):
    """d psi / d theta_j for every j, as an array [K, 2^n] (psi = branch state
    for Kraus indices k).  Product rule over the gates that use theta_j."""
    theta = np.asarray(theta, dtype=np.float64)
    out = np.zeros((circ.n_angles, 1 << circ.n), dtype=np.complex128)
    for j in range(circ.n_angles):
        for i, s in angle_gates(circ, j):
            op = circ.ops[i]
            a = s * theta[op[2]]
            dU = sim.dmat_rz(a) if op[0] == "RZ" else sim.dmat_rx(a)
            out[j] += s * sim.branch_state(circ, theta, k, noise, override={i: dU})
    return out


def expected_cost_param_shift(circ, theta, noise=None):
    """d<C>/d theta_j by the parameter-shift rule, <C> from the density matrix."""
    theta = np.asarray(theta, dtype=np.float64)
    g = np.zeros(circ.n_angles)
    for j in range(circ.n_angles):
        for i, s in angle_gates(circ, j):
            plus = sim.expected_cost(circ, theta, noise, shift={i: +np.pi / 2})
            minus = sim.expected_cost(circ, theta, noise, shift={i: -np.pi / 2})
            g[j] += s * 0.5 * (plus - minus)
    return g


def central_difference(fun, theta, h=1e-6):
    """Symmetric finite difference of a scalar or array-valued fun(theta)."""
    theta = np.asarray(theta, dtype=np.float64)
    cols = []
    for j in range(theta.size):
        tp = theta.copy()
        tm = theta.copy()
        tp.flat[j] += h
        tm.flat[j] -= h
        cols.append((np.asarray(fun(tp)) - np.asarray(fun(tm))) / (2 * h))
    return np.stack(cols)
