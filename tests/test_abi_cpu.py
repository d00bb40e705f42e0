"""The C ABI without a GPU: the library loads, exports exactly what
include/qkc.h declares, validates blobs before touching a device, and rejects
bad arguments with status codes (no compute calls are made here)."""
import ctypes
import os
import re
import struct

import numpy as np
import pytest

import workloads as W
from paper_2103_17226_amd import _lib as L
from paper_2103_17226_amd import blob as blobmod
from paper_2103_17226_amd import compiler as C

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_symbols():
    txt = open(os.path.join(ROOT, "include", "qkc.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(ac_[a-z_]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    lib = L.lib()
    declared = header_symbols()
    assert declared == sorted(L.EXPORTED)
    for name in declared:
        assert hasattr(lib, name), name


def _load(blob):
    h = ctypes.c_void_p()
    buf = ctypes.create_string_buffer(blob, len(blob))
    st = L.lib().ac_load(buf, len(blob), 0, ctypes.byref(h))
    return st, h


@pytest.fixture(scope="module")
def good_blob():
    return blobmod.to_blob(C.compile_circuit(W.config(1, small=True)["circuit"]))


def test_valid_blob_passes_format_checks(good_blob):
    st, h = _load(good_blob)
    # on a host without a GPU the first device query fails; on a GPU host it loads
    assert st in (L.AC_OK, L.AC_ERR_DEVICE), L.lib().ac_last_error()
    if st == L.AC_OK:
        L.lib().ac_free(h)


def test_corrupt_blobs_are_rejected_before_the_device(good_blob):
    b = bytearray(good_blob)
    bad_magic = bytes(b"XXXXXXXX" + b[8:])
    assert _load(bad_magic)[0] == L.AC_ERR_FORMAT
    assert _load(bytes(b[:40]))[0] == L.AC_ERR_FORMAT
    assert _load(bytes(b[:-16]))[0] == L.AC_ERR_FORMAT
    ver = bytearray(b)
    struct.pack_into("<I", ver, 8, 99)
    assert _load(bytes(ver))[0] == L.AC_ERR_FORMAT
    # corrupt the first child reference into a forward reference
    h = blobmod.blob_summary(good_blob)
    ac = C.compile_circuit(W.config(1, small=True)["circuit"])
    col = ac.col.copy()
    col[0] = np.uint32(ac.n_internal - 1)          # node 0 pointing at the root
    ac.col = col
    assert _load(blobmod.to_blob(ac))[0] == L.AC_ERR_FORMAT
    assert "not below" in L.lib().ac_last_error().decode()
    # bad slot reference, patched into the serialised col array
    def a8(x):
        return (x + 7) // 8 * 8
    nv, nn, S, N = h["n_vars"], h["n_noise"], h["n_slots"], h["n_int"]
    off = a8(64 + 2 * nv)
    off = a8(off + 4 * nv)
    off = a8(off + 8 * nn + 32 * S + 20 * h["n_selectors"] + N)
    off = a8(off + 4 * (N + 1))
    patched = bytearray(good_blob)
    struct.pack_into("<I", patched, off, (C.TAG_SLOT << C.TAG_SHIFT) | 999)
    assert _load(bytes(patched))[0] == L.AC_ERR_FORMAT
    assert "slot" in L.lib().ac_last_error().decode()
    # indicator value beyond the domain
    ac = C.compile_circuit(W.config(1, small=True)["circuit"])
    col = ac.col.copy()
    idx = int(np.nonzero((col >> C.TAG_SHIFT) == C.TAG_IND)[0][0])
    col[idx] = np.uint32(C.ref_ind(0, 3))
    ac.col = col
    assert _load(blobmod.to_blob(ac))[0] == L.AC_ERR_FORMAT


def test_null_arguments_are_rejected():
    lib = L.lib()
    assert lib.ac_free(None) == L.AC_OK
    assert lib.ac_info(None, None) == L.AC_ERR_INVALID_ARG
    assert lib.ac_workspace_size(None, 0, 10, 0) == 0
    assert lib.ac_workspace_size_share(None, 0, 10, 0, 0.5) == 0
    assert lib.ac_eval_batch(None, 0, None, 1, None, None, None, 1, None, None, None, 0, None) == L.AC_ERR_INVALID_ARG
    assert "null graph" in lib.ac_last_error().decode()
    assert lib.ac_grad_batch(None, 0, None, 1, None, None, None, 1, 0, None, None, None, None, None,
                             None, None, 0, None) == L.AC_ERR_INVALID_ARG
    cfg = L.SampleCfg(1, 1, 0, 1, 1, 0, 0, None)
    assert lib.ac_sample(None, 0, None, 1, None, ctypes.byref(cfg), None, None, None, None, None, 0,
                         None) == L.AC_ERR_INVALID_ARG
    h = ctypes.c_void_p()
    assert lib.ac_load(None, 0, 0, ctypes.byref(h)) == L.AC_ERR_INVALID_ARG
