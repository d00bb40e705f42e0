"""Serialise a compiled AC into the versioned binary blob that ``ac_load``
parses (layout documented in include/qkc.h).

Slots are reordered so that the angle-dependent ones come first; the
library evaluates those per batch element and the others once per call.
"""
from __future__ import annotations

import struct

import numpy as np

from .compiler import ANGLE_BASES, NO_SLOT, TAG_SHIFT, TAG_SLOT, CompiledAC

MAGIC = b"QKCAC\x00\x00\x01"
VERSION = 2
HEADER_FMT = "<8sIIIIIIIIIIIIII"     # magic + 14 u32
SLOT_FMT = "<BBHiddd"                # base, coef, pad, index, scale, re, im


def _align8(buf: bytearray):
    while len(buf) % 8:
        buf.append(0)


def to_blob(ac: CompiledAC) -> bytes:
    # angle slots first
    order = sorted(range(len(ac.slots)), key=lambda s: (0 if ac.slots[s].base in ANGLE_BASES else 1, s))
    remap = np.zeros(len(ac.slots), dtype=np.uint32)
    for new, old in enumerate(order):
        remap[old] = new
    slots = [ac.slots[o] for o in order]
    n_angle_slots = sum(1 for s in slots if s.base in ANGLE_BASES)
    col = ac.col.astype(np.uint32).copy()
    is_slot = (col >> TAG_SHIFT) == TAG_SLOT
    col[is_slot] = (np.uint32(TAG_SLOT) << np.uint32(TAG_SHIFT)) | remap[col[is_slot] & np.uint32((1 << TAG_SHIFT) - 1)]

    n_vars = len(ac.var_dom)
    hdr = struct.pack(HEADER_FMT, MAGIC, VERSION, 0, ac.n_qubits, n_vars, ac.n_words,
                      ac.n_angles, ac.n_noise, len(slots), n_angle_slots, ac.n_internal,
                      ac.n_edges, ac.n_levels, ac.root, len(ac.selectors))
    buf = bytearray(hdr)
    _align8(buf)
    buf += np.asarray(ac.var_dom, dtype=np.uint8).tobytes()
    buf += np.asarray(ac.var_kind, dtype=np.uint8).tobytes()
    _align8(buf)
    buf += np.asarray(ac.var_offset, dtype=np.uint32).tobytes()
    _align8(buf)
    buf += np.asarray(ac.noise_default, dtype=np.float64).tobytes()
    for s in slots:
        buf += struct.pack(SLOT_FMT, s.base, s.coef, 0, s.index, s.scale, s.re, s.im)
    for v, sl in ac.selectors:
        ent = [0xFFFFFFFF if x == NO_SLOT else int(remap[x]) for x in sl]
        ent += [0xFFFFFFFF] * (4 - len(ent))
        buf += struct.pack("<5I", v, *ent)
    buf += ac.op.astype(np.uint8).tobytes()
    _align8(buf)
    buf += ac.row_ptr.astype(np.uint32).tobytes()
    _align8(buf)
    buf += col.tobytes()
    _align8(buf)
    buf += ac.level_ptr.astype(np.uint32).tobytes()
    _align8(buf)
    return bytes(buf)


def blob_summary(blob: bytes) -> dict:
    f = struct.unpack_from(HEADER_FMT, blob, 0)
    keys = ["magic", "version", "flags", "n_qubits", "n_vars", "n_words", "n_angles", "n_noise",
            "n_slots", "n_angle_slots", "n_int", "n_edges", "n_levels", "root", "n_selectors"]
    return dict(zip(keys, f))


def compile_blob(circ, method: str = "ve", **kw) -> bytes:
    """Compile a circuit and serialise its AC (picklable entry point for
    compiling many circuits in worker processes).  method "ve" is variable
    elimination (compiler.compile_circuit), "dpll" the search-based compiler
    (dnnf.compile_circuit_dpll), "best" the smaller of the two; all give the
    same polynomial."""
    if method == "ve":
        from .compiler import compile_circuit
        return to_blob(compile_circuit(circ, **kw))
    if method == "dpll":
        from .dnnf import compile_circuit_dpll
        return to_blob(compile_circuit_dpll(circ, **kw))
    if method == "best":                   # both compilers; the AC with fewer internal nodes
        from .compiler import compile_circuit
        from .dnnf import compile_circuit_dpll
        ve, dp = compile_circuit(circ, **kw), compile_circuit_dpll(circ, **kw)
        return to_blob(dp if dp.n_internal < ve.n_internal else ve)
    raise ValueError(f"unknown compile method {method!r}")


def _compiler_key() -> str:
    """Hash of the compiler and blob writer sources (a cache entry is stale
    once either changes)."""
    import hashlib
    import os
    h = hashlib.sha256()
    here = os.path.dirname(os.path.abspath(__file__))
    for name in ("compiler.py", "dnnf.py", "blob.py"):
        with open(os.path.join(here, name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def compile_blob_cached(circ, cache_dir: str, **kw):
    """compile_blob with an on-disk cache keyed by the circuit (ops, noise
    strengths, size), the compile options and the compiler's source; returns
    (blob, cache hit).  An empty cache_dir disables the cache."""
    import hashlib
    import os
    import tempfile
    if not cache_dir:
        return compile_blob(circ, **kw), False
    key = hashlib.sha256(repr((circ.n, [tuple(op) for op in circ.ops], circ.n_angles,
                               [float(x) for x in circ.noise], sorted(kw.items()),
                               _compiler_key())).encode()).hexdigest()[:32]
    path = os.path.join(cache_dir, f"{key}.qkcac")
    try:
        with open(path, "rb") as f:
            blob = f.read()
        if blob[:8] == MAGIC:
            return blob, True
    except OSError:
        pass
    blob = compile_blob(circ, **kw)
    try:
        os.makedirs(cache_dir, exist_ok=True)
        fd, tmp = tempfile.mkstemp(dir=cache_dir)
        with os.fdopen(fd, "wb") as f:
            f.write(blob)
        os.replace(tmp, path)
    except OSError:
        pass
    return blob, False
