"""The allocation-free upward pass (ac_eval_batch_static) against
ac_eval_batch, both through the C ABI: the same kernels on the library's
static scratch instead of a caller workspace, so results must agree bit for
bit, on consecutive calls (the second with a smaller input), and with the
oracle (complex128 within 1e-12)."""
import ctypes

import numpy as np
import pytest
import torch

import workloads as W
from paper_2103_17226_amd import _lib as L
from tests.gpu_common import graph, note, oracle_amplitudes, require_gpu

pytestmark = pytest.mark.gpu


def _inputs(circ, P, B, seed):
    rng = np.random.default_rng(seed)
    theta = rng.uniform(0, 2 * np.pi, size=(P, circ.n_angles))
    vals = np.concatenate([rng.integers(0, 2, size=(B, circ.n)),
                           W.sample_channel_prior(circ, B, rng)], axis=1)
    return theta, vals, W.pack_evidence(circ, vals), (np.arange(B) % P).astype(np.int32)


def _static_call(g, dtype, theta, ev, po, want_prob=True):
    """ac_eval_batch_static through ctypes on caller-made tensors."""
    code, cdt = {"c64": (L.AC_C64, torch.complex64), "c128": (L.AC_C128, torch.complex128)}[dtype]
    dev = g.torch_device
    th = torch.as_tensor(theta, dtype=torch.float64, device=dev).contiguous()
    evt = torch.from_numpy(np.ascontiguousarray(ev).view(np.int64)).to(dev)
    pot = torch.as_tensor(po, dtype=torch.int32, device=dev)
    B = evt.shape[0]
    amp = torch.full((B,), complex(7.0, 7.0), dtype=cdt, device=dev)
    pr = torch.full((B,), -1.0, dtype=torch.float64, device=dev) if want_prob else None
    p = lambda t: ctypes.c_void_p(t.data_ptr()) if t is not None else None   # noqa: E731
    stream = ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)
    st = L.lib().ac_eval_batch_static(g._h, code, p(th), th.shape[0], None, p(pot), p(evt), B, p(amp), p(pr),
                                      stream)
    L.check(st)
    torch.cuda.synchronize()
    return amp.cpu().numpy(), (pr.cpu().numpy() if pr is not None else None)


@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_static_scratch_matches_workspace_call_twice_in_a_row(dtype):
    require_gpu()
    circ = W.qaoa_maxcut(6, W.random_regular_graph(6, 3, 4), 2, dep=0.02, ad=0.01)
    g = graph(circ)
    for call, (P, B, seed) in enumerate([(7, 1000, 11), (3, 131, 12)]):   # second call smaller
        note(f"static scratch {dtype} call {call}: P={P} B={B} nodes={g.info['n_internal']}")
        theta, vals, ev, po = _inputs(circ, P, B, seed)
        a_s, p_s = _static_call(g, dtype, theta, ev, po)
        a_w, p_w = g.eval(theta, ev, po, dtype=dtype)
        a_w, p_w = a_w.cpu().numpy(), p_w.cpu().numpy()
        assert np.array_equal(a_s.view(np.uint8), a_w.view(np.uint8))
        assert np.array_equal(p_s.view(np.uint8), p_w.view(np.uint8))
        if dtype == "c128":
            ref = np.concatenate([oracle_amplitudes(circ, theta[po[b]], vals[b:b + 1]) for b in range(0, B, 7)])
            assert np.max(np.abs(a_s[::7] - ref)) <= 1e-12


def test_static_scratch_caps_the_grid_on_a_large_graph_and_the_binding_agrees():
    require_gpu()
    # 12-qubit noisy p=2: tens of thousands of nodes, so the 256 MiB scratch
    # holds only some workgroups' rows and the grid is capped
    circ = W.qaoa_maxcut(12, W.random_regular_graph(12, 3, 5), 2, dep=0.01)
    g = graph(circ)
    N = g.info["n_internal"]
    note(f"static scratch capped grid: nodes={N}")
    for call, (P, B, seed) in enumerate([(16, 20000, 21), (5, 777, 22)]):
        theta, vals, ev, po = _inputs(circ, P, B, seed)
        a_s, p_s = _static_call(g, "c64", theta, ev, po)
        a_w, p_w = g.eval(theta, ev, po, dtype="c64")
        assert np.array_equal(a_s.view(np.uint8), a_w.cpu().numpy().view(np.uint8)), call
        assert np.array_equal(p_s.view(np.uint8), p_w.cpu().numpy().view(np.uint8)), call
    # the binding's method agrees too, and an empty batch enqueues nothing
    theta, vals, ev, po = _inputs(circ, 2, 64, 23)
    a_b, _ = g.eval_static(theta, ev, po, dtype="c128")
    a_w, _ = g.eval(theta, ev, po, dtype="c128")
    assert np.array_equal(a_b.cpu().numpy().view(np.uint8), a_w.cpu().numpy().view(np.uint8))
    a0, p0 = g.eval_static(theta, ev[:0], po[:0], dtype="c64")
    assert a0.numel() == 0


def _wide_sum_graph(M):
    """A one-qubit AC with M sum nodes on level 1, each holding the indicator
    [q0 = 0], and the root summing them on level 2: f = M [x0 = 0].  Its
    node rows are M + 1 per element, which sets how much scratch one tile
    takes without a long compile."""
    from paper_2103_17226_amd.compiler import TAG_IND, TAG_NODE, TAG_SHIFT, CompiledAC
    ind = np.uint32(TAG_IND << TAG_SHIFT)            # variable 0, value 0
    col = np.concatenate([np.full(M, ind, dtype=np.uint32),
                          (np.uint32(TAG_NODE << TAG_SHIFT) | np.arange(M, dtype=np.uint32))])
    row_ptr = np.concatenate([np.arange(M + 1, dtype=np.int64), [2 * M]]).astype(np.int32)
    return CompiledAC(n_qubits=1, var_dom=[2], var_kind=[0], var_offset=[0], n_words=1, n_angles=0,
                      n_noise=0, noise_default=[], slots=[], selectors=[],
                      op=np.zeros(M + 1, dtype=np.uint8), row_ptr=row_ptr, col=col,
                      level_ptr=np.array([0, M, M + 1], dtype=np.int32), root=M)


def test_static_scratch_one_workgroup_then_refusal_past_its_size():
    require_gpu()
    M = 300_000          # complex64 tile: 153.6 MB (fits once); complex128: 307 MB (does not)
    g = graph(_wide_sum_graph(M))
    note(f"static scratch wide-sum graph: nodes={g.info['n_internal']}")
    ev = np.array([[0], [1]] * 100, dtype=np.uint64)          # x0 = 0, 1, 0, 1, ...
    po = np.zeros(len(ev), dtype=np.int32)
    theta = np.zeros((1, 0))
    a_s, p_s = _static_call(g, "c64", theta, ev, po)
    a_w, _ = g.eval(theta, ev, po, dtype="c64")
    assert np.array_equal(a_s.view(np.uint8), a_w.cpu().numpy().view(np.uint8))
    want = np.where(ev[:, 0] == 0, float(M), 0.0)
    assert np.array_equal(a_s.real, want.astype(np.float32)) and not np.any(a_s.imag)
    with pytest.raises(L.ACError) as ei:
        _static_call(g, "c128", theta, ev, po)
    assert ei.value.status == L.AC_ERR_UNSUPPORTED and "static scratch" in str(ei.value)
