"""GPU parity of the most-probable-explanation query (ac_mpe_batch): for
every outcome x of small noisy circuits, the largest joint probability
max_k |f(x, k)|^2 against the oracle's enumeration of every Kraus branch
(complex128, 1e-12 relative), and the returned events must be one of the
maximisers (ties are common: X and Y errors often explain an outcome
equally well).  Batches span several 64-element tiles with a ragged tail."""
import numpy as np
import pytest

import workloads as W
from oracle import sim
from paper_2103_17226_amd import _lib as L
from paper_2103_17226_amd.compiler import compile_circuit
from paper_2103_17226_amd.dnnf import compile_circuit_dpll
from tests.gpu_common import graph, note, require_gpu
from tests.test_compiler import CIRCUITS

pytestmark = pytest.mark.gpu

NAMES = ["bell", "tiny", "ring3_dep", 0, 1, 2, 3, 4, 7, 8, 11]


@pytest.fixture(autouse=True)
def _gpu():
    require_gpu()


def _circ(name):
    return CIRCUITS[name]() if name in CIRCUITS else W.random_circuit(name)


@pytest.mark.parametrize("name", NAMES)
def test_mpe_matches_the_oracle_on_every_outcome(name):
    circ = _circ(name)
    g = graph(compile_circuit_dpll(circ, mpe=True))
    note(f"mpe {name}: {circ.n} qubits, {len(circ.channels())} channels, {g.info['n_internal']} nodes")
    rng = np.random.default_rng(40 + NAMES.index(name))
    P = 3
    theta = rng.uniform(0, 2 * np.pi, size=(P, circ.n_angles))
    B = 64 * 3 + 7
    xs = rng.integers(0, 1 << circ.n, size=B)
    po = rng.integers(0, P, size=B).astype(np.int32)
    doms = circ.var_domains()
    vals = np.zeros((B, len(doms)), dtype=np.int64)
    vals[:, :circ.n] = [[(x >> q) & 1 for q in range(circ.n)] for x in xs]
    for v in range(circ.n, len(doms)):                 # event fields in the input are ignored
        vals[:, v] = rng.integers(0, doms[v], size=B)
    prob, words = g.mpe(theta, W.pack_evidence(circ, vals), po)
    prob = prob.cpu().numpy()
    got = W.unpack_evidence(circ, words.cpu().numpy().view(np.uint64))
    cache = {}
    for b in range(B):
        key = (int(po[b]), int(xs[b]))
        if key not in cache:
            cache[key] = sim.most_probable_events(circ, theta[po[b]], int(xs[b]))
        best, ks = cache[key]
        assert abs(prob[b] - best) <= 1e-12 * max(best, 1e-300), (b, prob[b], best)
        assert np.array_equal(got[b, :circ.n], vals[b, :circ.n]), b
        if best > 0:
            assert tuple(int(k) for k in got[b, circ.n:]) in ks, (b, got[b, circ.n:], ks)


def test_mpe_with_a_noise_override_and_a_noise_free_circuit():
    circ = _circ("tiny")
    g = graph(compile_circuit_dpll(circ, mpe=True))
    noise = np.array(circ.noise) * 0.5 + 0.1
    theta = np.array([[0.4, 1.9]])
    xs = np.arange(1 << circ.n)
    vals = np.zeros((len(xs), len(circ.var_domains())), dtype=np.int64)
    vals[:, :circ.n] = [[(x >> q) & 1 for q in range(circ.n)] for x in xs]
    prob, _ = g.mpe(theta, W.pack_evidence(circ, vals), np.zeros(len(xs), np.int32), noise=noise)
    for x in xs:
        best, _ = sim.most_probable_events(circ, theta[0], int(x), noise=noise)
        assert abs(prob[int(x)].item() - best) <= 1e-12 * best
    # no channels: the most probable explanation is the outcome's own probability
    ring = W.config(1, small=True)["circuit"]
    g1 = graph(compile_circuit_dpll(ring, mpe=True))
    th = np.array([[0.3, 1.1]])
    vals = np.array([[(x >> q) & 1 for q in range(4)] for x in range(16)], dtype=np.int64)
    ev = W.pack_evidence(ring, vals)
    prob, words = g1.mpe(th, ev, np.zeros(16, np.int32))
    ref = np.abs(sim.statevector(ring, th[0])) ** 2
    assert np.max(np.abs(prob.cpu().numpy() - ref)) <= 1e-13
    assert np.array_equal(words.cpu().numpy().view(np.uint64), ev)


def test_mpe_refuses_acs_not_compiled_for_it():
    circ = _circ("tiny")
    theta = np.array([[0.4, 1.9]])
    vals = np.zeros((3, len(circ.var_domains())), dtype=np.int64)
    ev = W.pack_evidence(circ, vals)
    for ac in (compile_circuit(circ), compile_circuit_dpll(circ)):      # selector leaves
        g = graph(ac)
        with pytest.raises(L.ACError) as e:
            g.mpe(theta, ev, np.zeros(3, np.int32))
        assert e.value.status == L.AC_ERR_UNSUPPORTED and "selector" in str(e.value)
    g = graph(compile_circuit_dpll(circ, mpe=True))
    prob, words = g.mpe(theta, ev[:0], np.zeros(0, np.int32))          # an empty batch
    assert prob.numel() == 0 and words.shape[0] == 0
    # a parameter index outside [0, P) reads no parameters and gives NaN
    prob, _ = g.mpe(theta, ev, np.array([0, 1, -1], np.int32), validate=False)
    prob = prob.cpu().numpy()
    assert np.isfinite(prob[0]) and np.isnan(prob[1]) and np.isnan(prob[2])
    # complex128 only: the workspace query for another dtype is refused
    assert L.lib().ac_workspace_size(g._h, L.AC_C64, 3, L.AC_OP_MPE) == 0


def test_mpe_of_the_bench_circuit():
    # the bench's MPE workload (4-ring QAOA, 8 channels): sampled outcomes
    # and angle pairs against the oracle
    circ = W.qaoa_ring_mpe(4)
    g = graph(compile_circuit_dpll(circ, mpe=True))
    rng = np.random.default_rng(77)
    theta = rng.uniform(0, 2 * np.pi, size=(4, circ.n_angles))
    xs = np.tile(np.arange(16), 4)
    po = np.repeat(np.arange(4, dtype=np.int32), 16)
    vals = np.zeros((64, circ.n_vars), dtype=np.int64)
    vals[:, :4] = [[(x >> q) & 1 for q in range(4)] for x in xs]
    prob, words = g.mpe(theta, W.pack_evidence(circ, vals), po)
    prob = prob.cpu().numpy()
    got = W.unpack_evidence(circ, words.cpu().numpy().view(np.uint64))
    for b in range(0, 64, 9):
        best, ks = sim.most_probable_events(circ, theta[po[b]], int(xs[b]))
        assert abs(prob[b] - best) <= 1e-12 * best
        assert tuple(int(k) for k in got[b, 4:]) in ks


def test_mpe_is_the_same_for_every_launch_shape(monkeypatch):
    # tiles of 16 waves (two workgroups per CU, grid-stride rounds for large
    # batches) and of 4 waves give the same bits: every element is computed
    # by its own lane in a fixed order
    circ = W.qaoa_ring_mpe(4)
    ac = compile_circuit_dpll(circ, mpe=True)
    g = graph(ac)
    monkeypatch.setenv("QKC_TILE_WAVES", "4")
    g4 = graph(ac)
    monkeypatch.delenv("QKC_TILE_WAVES")
    rng = np.random.default_rng(5)
    P = 8
    theta = rng.uniform(0, 2 * np.pi, size=(P, circ.n_angles))
    big = 64 * 600
    xs = rng.integers(0, 16, size=big)
    po = rng.integers(0, P, size=big).astype(np.int32)
    vals = np.zeros((big, circ.n_vars), dtype=np.int64)
    vals[:, :4] = [[(x >> q) & 1 for q in range(4)] for x in xs]
    ev = W.pack_evidence(circ, vals)
    pb, wb = g.mpe(theta, ev, po)
    ps, wsm = g.mpe(theta, ev[:200], po[:200])
    assert np.array_equal(pb[:200].cpu().numpy(), ps.cpu().numpy())
    assert np.array_equal(wb[:200].cpu().numpy(), wsm.cpu().numpy())
    p4, w4 = g4.mpe(theta, ev, po)
    assert np.array_equal(pb.cpu().numpy(), p4.cpu().numpy())
    assert np.array_equal(wb.cpu().numpy(), w4.cpu().numpy())
