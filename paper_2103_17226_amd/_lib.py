"""ctypes view of the C ABI in include/qkc.h (argument marshalling only).

The shared library is built in-tree by ``paper_2103_17226_amd.build`` (or
``__graft_entry__.build()``).  There is no fallback: if the library is
missing, importing the entry points raises.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libqkc.so")

AC_OK, AC_ERR_INVALID_ARG, AC_ERR_FORMAT, AC_ERR_OOM, AC_ERR_DEVICE, AC_ERR_UNSUPPORTED = range(6)
STATUS_NAMES = {0: "AC_OK", 1: "AC_ERR_INVALID_ARG", 2: "AC_ERR_FORMAT", 3: "AC_ERR_OOM",
                4: "AC_ERR_DEVICE", 5: "AC_ERR_UNSUPPORTED"}
AC_C64, AC_C128 = 0, 1
AC_OP_EVAL, AC_OP_GRAD, AC_OP_SAMPLE, AC_OP_MPE = 0, 1, 2, 3
AC_GRAD_COTANGENT, AC_GRAD_PROB, AC_GRAD_LOGPROB = 0, 1, 2
AC_SAMPLER_STREAM, AC_SAMPLER_LDS, AC_SAMPLER_GLOBAL = 0, 1, 2

EXPORTED = ("ac_load", "ac_free", "ac_info", "ac_last_error", "ac_workspace_size", "ac_workspace_size_share",
            "ac_sample_shape",
            "ac_eval_batch", "ac_eval_batch_static", "ac_grad_batch", "ac_mpe_batch", "ac_sample")
AC_STATIC_SCRATCH_BYTES = 256 << 20


class ACInfo(ctypes.Structure):
    _fields_ = [("n_qubits", ctypes.c_int32), ("n_vars", ctypes.c_int32),
                ("n_words", ctypes.c_int32), ("n_angles", ctypes.c_int32),
                ("n_noise", ctypes.c_int32), ("n_slots", ctypes.c_int32),
                ("n_angle_slots", ctypes.c_int32), ("n_internal", ctypes.c_int32),
                ("n_edges", ctypes.c_int64), ("n_levels", ctypes.c_int32),
                ("max_level_width", ctypes.c_int32), ("n_indicator_leaves", ctypes.c_int32),
                ("root", ctypes.c_int32), ("device", ctypes.c_int32),
                ("n_prod_flops", ctypes.c_int64), ("n_selectors", ctypes.c_int32),
                ("n_super", ctypes.c_int32), ("n_super_levels", ctypes.c_int32),
                ("max_live", ctypes.c_int32), ("max_siblings", ctypes.c_int32),
                ("n_super_node_factors", ctypes.c_int64), ("n_super_down_reads", ctypes.c_int64),
                ("n_super_leaf_reads", ctypes.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class SampleCfg(ctypes.Structure):
    _fields_ = [("chains_per_param", ctypes.c_int32), ("samples_per_chain", ctypes.c_int32),
                ("burn_in_sweeps", ctypes.c_int32), ("thin_sweeps", ctypes.c_int32),
                ("seed", ctypes.c_uint64), ("n_cost_edges", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("cost_edges", ctypes.c_void_p),
                ("init_states", ctypes.c_void_p), ("first_sweep", ctypes.c_uint32),
                ("first_var", ctypes.c_uint32), ("chain_offset", ctypes.c_uint64)]


class ACError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


_lib = None


def lib():
    """Load libqkc.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2103_17226_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
    L.ac_load.argtypes = [vp, sz, ctypes.c_int, ctypes.POINTER(vp)]
    L.ac_load.restype = ctypes.c_int
    L.ac_free.argtypes = [vp]
    L.ac_free.restype = ctypes.c_int
    L.ac_info.argtypes = [vp, ctypes.POINTER(ACInfo)]
    L.ac_info.restype = ctypes.c_int
    L.ac_last_error.argtypes = []
    L.ac_last_error.restype = ctypes.c_char_p
    L.ac_workspace_size.argtypes = [vp, ctypes.c_int, i64, ctypes.c_int]
    L.ac_workspace_size.restype = sz
    L.ac_workspace_size_share.argtypes = [vp, ctypes.c_int, i64, ctypes.c_int, ctypes.c_double]
    L.ac_workspace_size_share.restype = sz
    L.ac_sample_shape.argtypes = [vp, ctypes.c_int, i64, ctypes.POINTER(i32), ctypes.POINTER(i64)]
    L.ac_sample_shape.restype = ctypes.c_int
    L.ac_eval_batch.argtypes = [vp, ctypes.c_int, vp, i32, vp, vp, vp, i64, vp, vp, vp, sz, vp]
    L.ac_eval_batch.restype = ctypes.c_int
    L.ac_eval_batch_static.argtypes = [vp, ctypes.c_int, vp, i32, vp, vp, vp, i64, vp, vp, vp]
    L.ac_eval_batch_static.restype = ctypes.c_int
    L.ac_grad_batch.argtypes = [vp, ctypes.c_int, vp, i32, vp, vp, vp, i64, ctypes.c_int, vp, vp,
                                vp, vp, vp, vp, vp, sz, vp]
    L.ac_grad_batch.restype = ctypes.c_int
    L.ac_mpe_batch.argtypes = [vp, vp, i32, vp, vp, vp, i64, vp, vp, vp, sz, vp]
    L.ac_mpe_batch.restype = ctypes.c_int
    L.ac_sample.argtypes = [vp, ctypes.c_int, vp, i32, vp, ctypes.POINTER(SampleCfg), vp, vp, vp,
                            vp, vp, sz, vp]
    L.ac_sample.restype = ctypes.c_int
    _lib = L
    return L


def check(status):
    if status != AC_OK:
        raise ACError(status, lib().ac_last_error().decode())
