"""ctypes binding of the plain CPU evaluator (include/qkc_cpu.h): the
baseline the GPU library is timed against.  Host arrays in, host arrays out;
it is separate from the GPU binding and never used by it."""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libqkc_cpu.so")
EXPORTED = ("qkc_cpu_load", "qkc_cpu_free", "qkc_cpu_last_error", "qkc_cpu_info", "qkc_cpu_eval",
            "qkc_cpu_sample")

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2103_17226_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
        L.qkc_cpu_load.argtypes = [vp, ctypes.c_size_t, ctypes.POINTER(vp)]
        L.qkc_cpu_free.argtypes = [vp]
        L.qkc_cpu_free.restype = None
        L.qkc_cpu_last_error.restype = ctypes.c_char_p
        L.qkc_cpu_info.argtypes = [vp] + [vp] * 6
        L.qkc_cpu_eval.argtypes = [vp, vp, i32, vp, vp, vp, i64, vp, ctypes.c_int]
        L.qkc_cpu_sample.argtypes = [vp, vp, i32, vp, i32, i32, i32, i32, ctypes.c_uint64, vp, vp, vp,
                                     ctypes.c_int]
        _lib = L
    return _lib


def _check(st):
    if st != 0:
        raise RuntimeError(lib().qkc_cpu_last_error().decode())


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


class CpuAC:
    """A compiled AC (blob bytes) on the host."""

    def __init__(self, blob: bytes):
        self._h = ctypes.c_void_p()
        buf = ctypes.create_string_buffer(blob, len(blob))
        _check(lib().qkc_cpu_load(buf, len(blob), ctypes.byref(self._h)))
        vals = [ctypes.c_int32(), ctypes.c_int64(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32(),
                ctypes.c_int32()]
        _check(lib().qkc_cpu_info(self._h, *[ctypes.byref(v) for v in vals]))
        self.n_internal, self.n_edges, self.n_vars, self.n_words, self.n_angles, self.n_qubits = \
            [v.value for v in vals]

    def close(self):
        if self._h.value:
            lib().qkc_cpu_free(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def eval(self, theta, evidence, param_of, noise=None, threads: int = 0) -> np.ndarray:
        theta = np.ascontiguousarray(theta, dtype=np.float64).reshape(-1, self.n_angles)
        ev = np.ascontiguousarray(evidence, dtype=np.uint64).reshape(-1, self.n_words)
        po = np.ascontiguousarray(param_of, dtype=np.int32)
        nz = None if noise is None else np.ascontiguousarray(noise, dtype=np.float64)
        out = np.empty((ev.shape[0], 2))
        _check(lib().qkc_cpu_eval(self._h, _p(theta), theta.shape[0], _p(nz), _p(po), _p(ev), ev.shape[0],
                                  _p(out), int(threads)))
        return out[:, 0] + 1j * out[:, 1]

    def sample(self, theta, chains_per_param: int, samples_per_chain: int = 1, burn_in: int = 10,
               thin: int = 1, seed: int = 1, noise=None, want_states: bool = False, threads: int = 0):
        theta = np.ascontiguousarray(theta, dtype=np.float64).reshape(-1, self.n_angles)
        P = theta.shape[0]
        S = chains_per_param * samples_per_chain
        samples = np.empty((P, S), dtype=np.uint64)
        states = np.empty((P, S, self.n_words), dtype=np.uint64) if want_states else None
        rounds = np.empty(P * chains_per_param, dtype=np.int64)
        nz = None if noise is None else np.ascontiguousarray(noise, dtype=np.float64)
        _check(lib().qkc_cpu_sample(self._h, _p(theta), P, _p(nz), int(chains_per_param), int(samples_per_chain),
                                    int(burn_in), int(thin), int(seed) & ((1 << 64) - 1), _p(samples),
                                    _p(states), _p(rounds), int(threads)))
        return dict(samples=samples, states=states, rounds=rounds)
