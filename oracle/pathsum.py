"""Python side of the brute-force QAOA p=1 path sum (see ``pathsum.c``).

Test infrastructure only (see ``oracle/__init__.py``).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pathsum.c")
_LIB = os.path.join(_HERE, "_pathsum.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile pathsum.c with gcc/OpenMP into oracle/_pathsum.so."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O3", "-fopenmp", "-shared", "-fPIC", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        lib.qkc_oracle_pathsum_hist.restype = ctypes.c_int
        lib.qkc_oracle_pathsum_hist.argtypes = [
            ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_uint64, ctypes.c_void_p]
        _lib = lib
    return _lib


def path_histogram(n, edges, x_index):
    """Exact integer counts H[cut, m] of paths z with cut(z)=cut and |z^x|=m."""
    lib = _load()
    e = np.ascontiguousarray(np.asarray(edges, dtype=np.int32).reshape(-1, 2))
    hist = np.zeros((len(e) + 1, n + 1), dtype=np.uint64)
    rc = lib.qkc_oracle_pathsum_hist(int(n), int(len(e)), e.ctypes.data, int(x_index),
                                     hist.ctypes.data)
    if rc != 0:
        raise RuntimeError(f"pathsum failed with code {rc}")
    return hist


def amplitudes_from_histogram(hist, n, n_edges, gammas, betas):
    """f(x) for each (gamma, beta) pair: sum over (cut, m) of the count times
    2^{-n/2} exp(-i g (|E| - 2 cut)) cos(b)^{n-m} (-i sin b)^m."""
    gammas = np.atleast_1d(np.asarray(gammas, dtype=np.float64))
    betas = np.atleast_1d(np.asarray(betas, dtype=np.float64))
    cuts = np.arange(hist.shape[0], dtype=np.float64)
    ms = np.arange(hist.shape[1])
    H = hist.astype(np.float64)
    out = np.zeros(len(gammas), dtype=np.complex128)
    for t, (g, b) in enumerate(zip(gammas, betas)):
        phase = np.exp(-1j * g * (n_edges - 2.0 * cuts))
        cb, sb = np.cos(b), -1j * np.sin(b)
        mix = np.array([cb ** (n - m) * sb ** m for m in ms])
        out[t] = (2.0 ** (-n / 2.0)) * np.sum(phase[:, None] * H * mix[None, :])
    return out


def qaoa_p1_amplitude(n, edges, x_index, gammas, betas):
    hist = path_histogram(n, edges, x_index)
    return amplitudes_from_histogram(hist, n, len(edges), gammas, betas)


def ring_amplitude(n, x_index, gamma, beta):
    """f(x) of noise-free QAOA p=1 on the n-ring (edges (i, i+1 mod n), n >= 3)
    at any n: the same closed path sum as above,
    f(x) = 2^{-n/2} sum_z prod_edges exp(-i g (1 - 2 [z_a != z_b])) prod_i R(x_i, z_i)
    with R(a, a) = cos b and R(a, not a) = -i sin b, summed over the paths z
    of the ring by transfer matrices: M_i[a][c] = R(x_i, a) exp(-i g (1 - 2 [a != c]))
    links z_i = a to z_{i+1} = c, and the sum is the trace of M_0 ... M_{n-1}.
    Exact in complex128 up to rounding; x_index holds bit i = x_i (n <= 64)."""
    if n < 3:
        raise ValueError("the ring needs n >= 3")
    x = int(x_index)
    cb, sb = np.cos(beta), -1j * np.sin(beta)
    bond = np.array([[np.exp(-1j * gamma), np.exp(1j * gamma)],
                     [np.exp(1j * gamma), np.exp(-1j * gamma)]])
    prod = np.eye(2, dtype=np.complex128)
    for i in range(n):
        xi = (x >> i) & 1
        r = np.array([cb if xi == 0 else sb, sb if xi == 0 else cb])   # R(x_i, z_i = 0 / 1)
        prod = prod @ (r[:, None] * bond)
    return complex(2.0 ** (-n / 2.0) * np.trace(prod))
