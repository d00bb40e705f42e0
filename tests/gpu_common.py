"""Shared helpers of the GPU tests (inputs from workloads, expectations from
the oracle; the GPU path is reached only through the C ABI binding)."""
import sys

import numpy as np
import pytest
import torch

from oracle import sim


def require_gpu():
    if not torch.cuda.is_available():
        pytest.fail("GPU test collected on a host without a HIP device")


def note(msg):
    print(f"[gpu-test] {msg}", flush=True)
    sys.stdout.flush()


def graph(circ, device=0):
    from paper_2103_17226_amd.api import ACGraph
    return ACGraph(circ, device=device)


def oracle_amplitudes(circ, theta, values, cache=None):
    """f(x, k) from Kraus-branch state vectors, values [B, n_vars]."""
    n = circ.n
    out = np.zeros(len(values), dtype=np.complex128)
    cache = {} if cache is None else cache
    th = np.asarray(theta, dtype=np.float64)
    for b, v in enumerate(values):
        key = (th.tobytes(), tuple(int(z) for z in v[n:]))
        vec = cache.get(key)
        if vec is None:
            vec = sim.branch_state(circ, th, v[n:])
            cache[key] = vec
        x = sum(int(v[q]) << q for q in range(n))
        out[b] = vec[x]
    return out


def prob_ok(p_gpu, p_ref, rel=1e-5):
    """Outcome-probability rule: relative error <= rel where the reference
    is at least 1e-3 of the largest probability in the set, absolute error
    <= rel * max elsewhere."""
    p_gpu = np.asarray(p_gpu, dtype=np.float64)
    p_ref = np.asarray(p_ref, dtype=np.float64)
    pmax = max(float(np.max(np.abs(p_ref))), 1e-300)
    big = p_ref >= 1e-3 * pmax
    err = np.abs(p_gpu - p_ref)
    ok_big = np.all(err[big] <= rel * p_ref[big])
    ok_small = np.all(err[~big] <= rel * pmax)
    return bool(ok_big and ok_small), float(np.max(err[big] / p_ref[big])) if big.any() else 0.0
