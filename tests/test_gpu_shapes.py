"""Results do not depend on the launch shape the library picks per call:
amplitudes, gradients and Gibbs chains are bit for bit the same with 4, 8
or 16 waves per 64-element tile (upward pass, gradients, streaming sampler),
with 1 to 16 waves per streaming tile, and with one or four waves per chain
in the LDS-resident sampler.  Each node is computed by one lane in a fixed
order whichever wave holds it, and every reduction has a fixed order."""
import numpy as np
import pytest
import torch

import workloads as W
from tests.gpu_common import graph, note, require_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _gpu():
    require_gpu()


def _inputs(circ, B, seed):
    rng = np.random.default_rng(seed)
    vals = np.concatenate([rng.integers(0, 2, size=(B, circ.n)), W.sample_channel_prior(circ, B, rng)], axis=1)
    theta = rng.uniform(0, 2 * np.pi, size=(3, circ.n_angles))
    po = rng.integers(0, 3, size=B).astype(np.int32)
    return theta, W.pack_evidence(circ, vals), po, rng.uniform(0.5, 2.0, size=B)


@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_tile_kernels_same_results_for_every_workgroup_size(dtype, monkeypatch):
    note(f"upward pass and gradients across 4 / 8 / 16 waves per tile ({dtype})")
    circ = W.config(2, small=True)["circuit"]
    theta, ev, po, w = _inputs(circ, 64 * 10 + 17, 5)
    ref = None
    for waves in ("4", "8", "16"):
        monkeypatch.setenv("QKC_TILE_WAVES", waves)
        g = graph(circ)                       # the size is read when the graph is loaded
        amp, prob = g.eval(theta, ev, po, dtype=dtype)
        out = g.grad(theta, ev, po, mode="prob", weight=w, dtype=dtype)
        got = (amp.cpu(), prob.cpu(), out["grad"].cpu())
        if ref is None:
            ref = got
        else:
            assert all(torch.equal(a, b) for a, b in zip(got, ref)), waves
        g.close()


def test_streaming_sampler_same_chains_for_every_workgroup_size(monkeypatch):
    note("streaming sampler across 1 to 16 waves per tile")
    circ = W.config(2, small=True)["circuit"]
    theta = np.array([[0.7, 0.4], [2.2, 1.3]])
    monkeypatch.setenv("QKC_SAMPLE_KERNEL", "stream")
    ref = None
    for waves in ("1", "2", "4", "8", "16"):
        monkeypatch.setenv("QKC_STREAM_WAVES", waves)
        g = graph(circ)
        out = g.sample(theta, 100, 2, 3, 1, 99, dtype="c128", want_states=True, want_rounds=True)
        got = (out["states"].cpu(), out["rounds"].cpu())
        if ref is None:
            ref = got
        else:
            assert torch.equal(got[0], ref[0]) and torch.equal(got[1], ref[1]), waves
        g.close()


@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_lds_sampler_same_chains_on_one_or_four_waves(dtype, monkeypatch):
    note(f"LDS-resident sampler, one or four waves per chain ({dtype})")
    circ = W.config(2, small=True)["circuit"]
    g = graph(circ)
    theta = np.array([[0.7, 0.4], [2.2, 1.3]])
    monkeypatch.setenv("QKC_SAMPLE_KERNEL", "lds")
    monkeypatch.setenv("QKC_SAMPLE_CPW", "1")
    outs = []
    for wpc in ("1", "4"):
        monkeypatch.setenv("QKC_SAMPLE_WPC", wpc)
        out = g.sample(theta, 150, 2, 3, 1, 7, dtype=dtype, want_states=True, want_rounds=True)
        outs.append((out["states"].cpu(), out["rounds"].cpu()))
    assert torch.equal(outs[0][0], outs[1][0]) and torch.equal(outs[0][1], outs[1][1])


def test_a_smaller_workspace_runs_fewer_workgroups_with_the_same_results():
    # the grid shrinks to the per-workgroup regions the workspace holds; each
    # element and chain is computed alone, so results do not change
    from paper_2103_17226_amd import _lib as L
    note("eval, gradients and both row-buffer samplers with 1/2, 1/7 and one workgroup's workspace")
    circ = W.config(2, small=True)["circuit"]
    g = graph(circ)
    theta, ev, po, w = _inputs(circ, 64 * 9 + 5, 8)
    B = ev.shape[0]

    def sizes(op, batch):
        full = g.workspace_size("c64", batch, op)
        return [full, full // 2, full // 7]
    ref = None
    for n in sizes(L.AC_OP_EVAL, B):
        ws = torch.empty(n, dtype=torch.uint8, device="cuda")
        amp, prob = g.eval(theta, ev, po, dtype="c64", ws=ws)
        got = (amp.cpu(), prob.cpu())
        ref = got if ref is None else ref
        assert all(torch.equal(a, b) for a, b in zip(got, ref)), n
    ref = None
    for n in sizes(L.AC_OP_GRAD, B):
        ws = torch.empty(n, dtype=torch.uint8, device="cuda")
        out = g.grad(theta, ev, po, mode="prob", weight=w, dtype="c64", ws=ws)
        got = out["grad"].cpu()
        ref = got if ref is None else ref
        assert torch.equal(got, ref), n
    th = np.array([[0.7, 0.4], [2.2, 1.3], [0.1, 2.9]])
    for kernel in ("stream", "global"):
        import os
        os.environ["QKC_SAMPLE_KERNEL"] = kernel
        try:
            gk = graph(circ)
            ref = None
            full = gk.workspace_size("c64", 3 * 400, L.AC_OP_SAMPLE)
            for n in (full, full // 2, full // 7):
                ws = torch.empty(n, dtype=torch.uint8, device="cuda")
                out = gk.sample(th, 400, 1, 3, 1, 17, dtype="c64", want_states=True, want_rounds=True, ws=ws)
                got = (out["samples"].cpu(), out["states"].cpu(), out["rounds"].cpu())
                ref = got if ref is None else ref
                assert all(torch.equal(a, b) for a, b in zip(got, ref)), (kernel, n)
            gk.close()
        finally:
            del os.environ["QKC_SAMPLE_KERNEL"]
    too_small = torch.empty(256, dtype=torch.uint8, device="cuda")
    with pytest.raises(L.ACError):
        g.eval(theta, ev, po, dtype="c64", ws=too_small)
    # ac_workspace_size_share: a share of the full-width workspace, the full
    # size at share 1, refused outside (0, 1]
    for op, batch in ((L.AC_OP_EVAL, B), (L.AC_OP_GRAD, B)):
        full = g.workspace_size("c64", batch, op)
        half = g.workspace_size_share("c64", batch, op, 0.5)
        assert half < full and g.workspace_size_share("c64", batch, op, 1.0) == full
        ws = torch.empty(half, dtype=torch.uint8, device="cuda")
        if op == L.AC_OP_EVAL:
            amp, _ = g.eval(theta, ev, po, dtype="c64", ws=ws)
        for bad in (0.0, -0.5, 1.5, float("nan")):
            with pytest.raises(L.ACError):
                g.workspace_size_share("c64", batch, op, bad)
    g.close()
