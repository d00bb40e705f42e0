"""Host logic of the request loop: admission by memory, arrival order,
merging, stream limits, cancellation, failures and latency bookkeeping.

The device is replaced by an executor written here, driven by a clock the
test advances, so every decision of the scheduler is checked on the CPU.
"""
import threading
import time
from concurrent.futures import CancelledError

import numpy as np
import pytest

from paper_2103_17226_amd.serve import (GRAD_ALIGN, AdmissionError, Request, Server, padded_rows,
                                        stack_eval_batch)


class Clock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t


class FakeExecutor:
    """Requests carry their footprint and latency in ``theta``'s first entries
    ([footprint, latency, value]); the result of a request is value * 2."""

    def __init__(self, clock, n_streams=4, fail_launch=(), fail_results=(), fail_done=()):
        self.clock = clock
        self.n_streams = n_streams
        self.launched = []                # (rids, stream, time)
        self.fail_launch = set(fail_launch)
        self.fail_results = set(fail_results)
        self.fail_done = set(fail_done)
        self.live_streams = set()

    def footprint(self, req):
        return int(req.theta[0, 0])

    def cost(self, req):
        return float(req.theta[0, 1])

    def can_merge(self, a, b):
        return a.kind == b.kind == "eval" and a.graph == b.graph and a.grad == b.grad and a.dtype == b.dtype

    def launch(self, batch, stream):
        assert stream not in self.live_streams, "stream reused while busy"
        if any(float(r.theta[0, 2]) in self.fail_launch for r in batch):
            raise RuntimeError("launch failed")
        self.live_streams.add(stream)
        lat = max(float(r.theta[0, 1]) for r in batch)
        self.launched.append(([r.rid for r in batch], stream, self.clock()))
        return {"end": self.clock() + lat, "batch": batch, "stream": stream}

    def done(self, h):
        ok = self.clock() >= h["end"]
        if ok:
            self.live_streams.discard(h["stream"])
            if any(float(r.theta[0, 2]) in self.fail_done for r in h["batch"]):
                raise RuntimeError("device error")
        return ok

    def results(self, h):
        if any(float(r.theta[0, 2]) in self.fail_results for r in h["batch"]):
            raise RuntimeError("copy-back failed")
        return [float(r.theta[0, 2]) * 2 for r in h["batch"]]


def req(fp, lat, val=1.0, graph="g", samples=1, grad=False, session=None):
    return Request(graph=graph, theta=np.array([[fp, lat, val]]), samples=samples, grad=grad, session=session)


def ev_req(fp, lat, val=1.0, graph="g", grad=False):
    return Request(graph=graph, theta=np.array([[fp, lat, val]]), evidence=np.zeros((1, 1), np.uint64),
                   grad=grad)


def run_until_idle(srv, clock, dt=0.5, limit=1000):
    for _ in range(limit):
        srv.step()
        if srv.idle():
            return
        clock.t += dt
    raise AssertionError("scheduler did not drain")


def test_admission_never_exceeds_budget():
    clock = Clock()
    ex = FakeExecutor(clock, n_streams=8)
    srv = Server(ex, mem_budget=100, clock=clock)
    futs = [srv.submit(req(40, 1.0, val=i)) for i in range(5)]
    srv.step()
    assert srv.used == 80 and len(ex.launched) == 2          # third does not fit yet
    clock.t = 1.0
    srv.step()
    assert [f.result() for f in futs[:2]] == [0.0, 2.0]
    assert len(ex.launched) == 4 and srv.used == 80
    run_until_idle(srv, clock)
    assert [f.result() for f in futs] == [2.0 * i for i in range(5)]
    assert srv.peak_used == 80 and srv.used == 0


def test_arrival_order_head_is_never_overtaken():
    clock = Clock()
    ex = FakeExecutor(clock, n_streams=8)
    srv = Server(ex, mem_budget=100, clock=clock)
    srv.submit(req(60, 1.0, val=1))
    srv.submit(req(60, 1.0, val=2))
    srv.submit(req(10, 1.0, val=3))          # would fit next to the first, but must wait
    srv.step()
    assert [x[0] for x in ex.launched] == [[0]]
    clock.t = 1.0
    srv.step()
    assert [x[0] for x in ex.launched] == [[0], [1], [2]]


def test_oversized_and_queue_full_are_rejected():
    clock = Clock()
    srv = Server(FakeExecutor(clock), mem_budget=100, clock=clock, max_queue=2)
    f = srv.submit(req(101, 1.0))
    with pytest.raises(AdmissionError):
        f.result(timeout=0)
    srv.submit(req(10, 1.0))
    srv.submit(req(10, 1.0))
    f3 = srv.submit(req(10, 1.0))
    with pytest.raises(AdmissionError, match="queue full"):
        f3.result(timeout=0)
    assert srv.rejected_memory == 1 and srv.rejected_queue == 1
    run_until_idle(srv, clock)
    assert srv.latency_stats()["completed"] == 2


def test_time_limit_rejects_long_requests():
    clock = Clock()
    srv = Server(FakeExecutor(clock), mem_budget=100, clock=clock, max_seconds=5.0)
    f = srv.submit(req(10, 6.0))
    ok = srv.submit(req(10, 4.0, val=3))
    with pytest.raises(AdmissionError, match="hold the device"):
        f.result(timeout=0)
    run_until_idle(srv, clock)
    assert ok.result() == 6.0 and srv.latency_stats()["rejected_cost"] == 1


def test_streams_bound_the_launches_in_flight():
    clock = Clock()
    ex = FakeExecutor(clock, n_streams=2)
    srv = Server(ex, mem_budget=10 ** 6, clock=clock)
    futs = [srv.submit(req(1, 1.0, val=i)) for i in range(5)]
    srv.step()
    assert len(srv.inflight) == 2
    run_until_idle(srv, clock)
    assert srv.max_inflight == 2 and all(f.done() for f in futs)


def test_eval_requests_of_one_graph_merge_others_do_not():
    clock = Clock()
    ex = FakeExecutor(clock, n_streams=4)
    srv = Server(ex, mem_budget=10 ** 6, clock=clock, max_merge=3)
    fa = [srv.submit(ev_req(1, 1.0, val=i, graph="a")) for i in range(2)]
    fb = srv.submit(ev_req(1, 1.0, val=9, graph="b"))
    fa += [srv.submit(ev_req(1, 1.0, val=i, graph="a")) for i in range(2, 5)]
    fg = srv.submit(ev_req(1, 1.0, val=7, graph="a", grad=True))
    fs = srv.submit(req(1, 1.0, val=8, graph="a"))             # a sampling request: alone
    srv.step()
    batches = [x[0] for x in ex.launched]
    assert batches == [[0, 1, 3], [2], [4, 5], [6]]
    srv.step()
    run_until_idle(srv, clock)
    assert [f.result() for f in fa] == [0.0, 2.0, 4.0, 6.0, 8.0]
    assert fb.result() == 18.0 and fg.result() == 14.0 and fs.result() == 16.0
    assert sorted(sum((x[0] for x in ex.launched), [])) == list(range(8))
    assert srv.merged == 3


def test_requests_of_one_session_run_one_at_a_time():
    clock = Clock()
    ex = FakeExecutor(clock, n_streams=4)
    srv = Server(ex, mem_budget=1000, clock=clock)
    a1 = srv.submit(req(10, 2.0, val=1, session="s"))
    a2 = srv.submit(req(10, 1.0, val=2, session="s"))
    b = srv.submit(req(10, 1.0, val=3, session="t"))
    c = srv.submit(req(10, 1.0, val=4))
    srv.step()
    assert [x[0] for x in ex.launched] == [[0], [2], [3]]        # a2 waits for a1, others go ahead
    clock.t = 1.0
    srv.step()
    assert len(ex.launched) == 3
    clock.t = 2.0
    srv.step()
    assert [x[0] for x in ex.launched][-1] == [1]
    run_until_idle(srv, clock)
    assert [f.result() for f in (a1, a2, b, c)] == [2.0, 4.0, 6.0, 8.0]
    assert not srv.busy_sessions


def test_resident_session_bytes_count_against_the_budget():
    clock = Clock()
    ex = FakeExecutor(clock, n_streams=4)
    ex.resident = 50
    ex.resident_bytes = lambda: ex.resident
    srv = Server(ex, mem_budget=100, clock=clock)
    f1 = srv.submit(req(40, 1.0))
    f2 = srv.submit(req(40, 1.0))
    srv.step()
    assert len(ex.launched) == 1                 # 50 resident + 40 + 40 > 100
    ex.resident = 0
    run_until_idle(srv, clock)
    assert f1.done() and f2.done()


def test_request_timeout_fails_the_caller_but_holds_resources_until_done():
    clock = Clock()
    ex = FakeExecutor(clock, n_streams=1)
    srv = Server(ex, mem_budget=100, clock=clock, request_timeout=5.0)
    slow = srv.submit(req(60, 10.0, val=1))
    nxt = srv.submit(req(60, 1.0, val=2))
    srv.step()
    clock.t = 6.0
    srv.step()
    with pytest.raises(TimeoutError):
        slow.result(timeout=0)
    assert srv.used == 60 and not nxt.done()      # the kernel still holds its memory and stream
    clock.t = 10.0
    srv.step()
    assert srv.used == 60 and not nxt.done()      # the next one started
    run_until_idle(srv, clock)
    assert nxt.result() == 4.0 and srv.latency_stats()["timed_out"] == 1


def test_cancel_waiting_but_not_running():
    clock = Clock()
    srv = Server(FakeExecutor(clock, n_streams=1), mem_budget=100, clock=clock)
    f0 = srv.submit(req(10, 1.0, val=1))
    f1 = srv.submit(req(10, 1.0, val=2))
    srv.step()
    assert not srv.cancel(f0)                 # already on the device
    assert srv.cancel(f1)
    with pytest.raises(CancelledError):
        f1.result(timeout=0)
    run_until_idle(srv, clock)
    assert f0.result() == 2.0 and srv.cancelled == 1


@pytest.mark.parametrize("where", ["launch", "done", "results"])
def test_failures_fail_the_batch_and_free_resources(where):
    clock = Clock()
    kw = {"fail_" + where: {5.0}}
    ex = FakeExecutor(clock, n_streams=1, **kw)
    srv = Server(ex, mem_budget=100, clock=clock)
    bad = srv.submit(req(60, 1.0, val=5.0))
    good = srv.submit(req(60, 1.0, val=1.0))
    run_until_idle(srv, clock)
    with pytest.raises(RuntimeError):
        bad.result(timeout=0)
    assert good.result() == 2.0
    assert srv.used == 0 and srv.free_streams == [0] and srv.failed == 1


def test_latency_percentiles_and_warmup_window():
    clock = Clock()
    srv = Server(FakeExecutor(clock, n_streams=100), mem_budget=10 ** 6, clock=clock)
    for i in range(100):
        clock.t = float(i)
        srv.submit(req(1, 0.0 if i < 10 else float(i - 9), val=i))
        srv.step()
    run_until_idle(srv, clock, dt=0.25)
    st = srv.latency_stats(since=10.0)
    assert st["completed"] == 90
    lat = np.array([r.t_done - r.t_arrive for r in srv.completed if r.t_arrive >= 10.0])
    assert st["p50_ms"] == pytest.approx(np.percentile(lat, 50) * 1e3)
    assert st["p99_ms"] == pytest.approx(np.percentile(lat, 99) * 1e3)
    # completions are seen at the first tick at or after the device finishes
    assert np.all(lat >= np.arange(1, 91) - 1e-9) and np.all(lat <= np.arange(1, 91) + 0.25 + 1e-9)


def test_threaded_loop_serves_concurrent_clients():
    ex = FakeExecutor(time.perf_counter, n_streams=4)
    srv = Server(ex, mem_budget=1000, clock=time.perf_counter)
    srv.start()
    out = {}

    def client(c):
        futs = []
        for i in range(50):
            r = ev_req(30, 1e-3, val=c * 100 + i, graph=f"g{c % 2}") if i % 3 else req(30, 2e-3, val=c * 100 + i)
            futs.append((c * 100 + i, srv.submit(r)))
            time.sleep(1e-4)
        out[c] = [(v, f.result(timeout=30)) for v, f in futs]

    th = [threading.Thread(target=client, args=(c,)) for c in range(4)]
    for t in th:
        t.start()
    for t in th:
        t.join(60)
    srv.stop()
    for c in range(4):
        assert [2.0 * v for v, _ in out[c]] == [r for _, r in out[c]]
    st = srv.latency_stats()
    assert st["completed"] == 200 and st["failed"] == 0 and srv.used == 0


def test_stop_waits_for_a_launch_in_progress():
    # a batch taken from the queue but still inside launch() keeps the loop busy
    started, release = threading.Event(), threading.Event()

    class SlowLaunch(FakeExecutor):
        def launch(self, batch, stream):
            started.set()
            release.wait(5)
            return super().launch(batch, stream)

    ex = SlowLaunch(time.perf_counter, n_streams=1)
    srv = Server(ex, mem_budget=100, clock=time.perf_counter)
    srv.start()
    f = srv.submit(req(10, 1e-3, val=4))
    assert started.wait(5)
    assert not srv.idle()
    threading.Timer(0.05, release.set).start()
    srv.stop(drain=True, timeout=10)
    assert f.result(timeout=0) == 8.0


def test_stop_without_drain_cancels_waiting():
    clock = Clock()
    srv = Server(FakeExecutor(clock, n_streams=1), mem_budget=100, clock=clock)
    srv.start()
    f0 = srv.submit(req(10, 1e9))
    f1 = srv.submit(req(10, 1.0))
    time.sleep(0.05)
    srv.stop(drain=False)
    assert f1.cancelled() and not f0.done()


# ------------------------------------------------------------- batch stacking

def _eval_request(rng, P, B, K=2, W=3, grad=True):
    return Request(graph="g", theta=rng.uniform(0, 6, size=(P, K)),
                   evidence=rng.integers(0, 1 << 62, size=(B, W), dtype=np.uint64),
                   param_of=rng.integers(0, P, size=B).astype(np.int32),
                   weight=rng.normal(size=B), grad=grad)


@pytest.mark.parametrize("grad", [False, True])
def test_stacked_batch_keeps_every_request_intact(grad):
    rng = np.random.default_rng(4)
    batch = [_eval_request(rng, P, B, grad=grad) for P, B in [(3, 5), (1, 256), (7, 300), (2, 0), (4, 64)]]
    theta, ev, po, wt, spans = stack_eval_batch(batch, 2, 3, grad)
    assert len(po) == len(ev) == sum(padded_rows(r.n_rows, grad) for r in batch)
    extra = 1 if grad else 0
    assert theta.shape == (sum(r.n_params for r in batch) + extra, 2)
    for r, (p0, P, b0, B) in zip(batch, spans):
        assert (P, B) == (r.n_params, r.n_rows)
        if grad:
            assert b0 % GRAD_ALIGN == 0
        np.testing.assert_array_equal(theta[p0:p0 + P], r.theta)
        np.testing.assert_array_equal(ev[b0:b0 + B], r.evidence)
        np.testing.assert_array_equal(po[b0:b0 + B], r.param_of + p0)
        if grad:
            np.testing.assert_array_equal(wt[b0:b0 + B], r.weight)
    covered = np.zeros(len(po), bool)
    for p0, P, b0, B in spans:
        covered[b0:b0 + B] = True
    if grad:
        # padding rows: weight 0, the extra all-zero parameter row
        assert np.all(wt[~covered] == 0) and np.all(po[~covered] == theta.shape[0] - 1)
        assert np.all(theta[-1] == 0)
    else:
        assert covered.all() and wt is None


def test_stacking_rejects_bad_param_rows():
    rng = np.random.default_rng(1)
    r = _eval_request(rng, 2, 4)
    r.param_of = np.array([0, 1, 2, 0], np.int32)
    with pytest.raises(ValueError):
        stack_eval_batch([r], 2, 3, True)


# ---------------------------------------------------------------------------
# split requests, resident sessions, the sampled-gradient estimator
# ---------------------------------------------------------------------------

class SplitExecutor(FakeExecutor):
    """FakeExecutor whose requests carry k units of work in ``samples``
    (cost = 1 s per unit): split() cuts them into parts of at most
    floor(limit) units; a part's result is the list of its units' values."""

    def cost(self, req):
        return float(req.samples)

    def split(self, req, limit, max_bytes=None):
        k = int(limit)
        if k < 1:
            return None
        out = []
        for u0 in range(0, req.samples, k):
            u1 = min(req.samples, u0 + k)
            out.append(Request(graph=req.graph, theta=req.theta, samples=u1 - u0, part=(u0, u1)))
        return out

    def launch(self, batch, stream):
        h = super().launch(batch, stream)
        h["end"] = self.clock() + max(float(r.samples) for r in batch)
        self.kinds = getattr(self, "kinds", []) + [(r.parent is not None, stream, r.share) for r in batch]
        return h

    def results(self, h):
        super().results(h)                       # the failures FakeExecutor injects
        out = []
        for r in h["batch"]:
            u0, u1 = r.part[1] if r.parent is not None else (0, r.samples)
            out.append([float(r.theta[0, 2]) + u for u in range(u0, u1)])
        return out

    def combine(self, req, outs):
        return sum(outs, [])


def test_requests_over_the_time_limit_are_split_and_reassembled():
    clock = Clock()
    ex = SplitExecutor(clock, n_streams=2)
    srv = Server(ex, mem_budget=1000, clock=clock, max_seconds=3.0)
    big = srv.submit(req(10, 0.0, val=100, samples=8))        # 8 units -> parts of 3, 3, 2
    small = srv.submit(req(10, 0.0, val=7, samples=2))
    run_until_idle(srv, clock)
    assert big.result() == [100.0 + u for u in range(8)]
    assert small.result() == [7.0, 8.0]
    st = srv.latency_stats()
    assert st["rejected_cost"] == 0 and st["split_requests"] == 1 and st["split_parts"] == 3
    assert st["completed"] == 2                                 # parts are not requests of their own
    done = {r.rid: r for r in srv.completed}
    assert all(r.t_done >= r.t_arrive for r in done.values())


def test_a_split_request_fails_once_when_a_part_fails():
    clock = Clock()
    ex = SplitExecutor(clock, n_streams=4, fail_results={5.0})
    srv = Server(ex, mem_budget=1000, clock=clock, max_seconds=2.0)
    bad = srv.submit(req(10, 0.0, val=5.0, samples=5))
    ok = srv.submit(req(10, 0.0, val=1.0, samples=1))
    run_until_idle(srv, clock)
    with pytest.raises(RuntimeError):
        bad.result(timeout=0)
    assert ok.result() == [1.0] and srv.failed == 1


def test_idle_sessions_are_released_when_they_block_the_queue():
    # resident session bytes never shrink on their own: with nothing in
    # flight the head of the queue releases idle sessions, least recently
    # used first, and a request that cannot fit even then fails instead of
    # blocking every request behind it
    clock = Clock()
    ex = FakeExecutor(clock, n_streams=4)
    ex.sess = {("g", "old"): (30, 0), ("g", "new"): (30, 1), ("g", "busy"): (30, 2)}
    ex.resident_bytes = lambda: sum(b for b, _ in ex.sess.values())

    def evict(need, busy):
        n = 0
        for k, _ in sorted(ex.sess.items(), key=lambda kv: kv[1][1]):
            if need <= 0:
                break
            if k in busy:
                continue
            need -= ex.sess.pop(k)[0]
            n += 1
        return n
    ex.evict_sessions = evict
    srv = Server(ex, mem_budget=100, clock=clock)
    srv.busy_sessions.add(("g", "busy"))
    f1 = srv.submit(req(35, 1.0, val=1))          # needs one session released: the oldest
    f2 = srv.submit(req(80, 1.0, val=2))          # cannot fit next to the busy session: fails
    f3 = srv.submit(req(10, 1.0, val=3))
    run_until_idle(srv, clock)
    assert f1.result() == 2.0 and f3.result() == 6.0
    with pytest.raises(AdmissionError, match="resident"):
        f2.result(timeout=0)
    assert ("g", "old") not in ex.sess and ("g", "busy") in ex.sess
    assert srv.evicted_sessions >= 1 and srv.rejected_memory == 1


def test_sampled_gradient_needs_two_samples():
    clock = Clock()
    srv = Server(FakeExecutor(clock), mem_budget=100, clock=clock)
    f = srv.submit(req(10, 1.0, samples=1, grad=True))
    with pytest.raises(AdmissionError, match="at least 2"):
        f.result(timeout=0)
    assert srv.rejected_invalid == 1


@pytest.mark.parametrize("S", [2, 3])
def test_leave_one_out_score_gradient_is_unbiased(S):
    # The estimator's mean over every ordered S-tuple of draws from a small
    # discrete law p(x) with scores g(x) = d log p / d theta (so E[g] = 0)
    # equals the exact gradient sum_x p(x) C(x) g(x); the mean-over-all-S
    # baseline misses it by the factor (1 - 1/S).
    import itertools as it

    from paper_2103_17226_amd.serve import loo_score_gradient
    rng = np.random.default_rng(S)
    n, K = 4, 2
    th = rng.normal(size=(n, K))
    a = rng.normal(size=K)
    logits = th @ a
    p = np.exp(logits) / np.exp(logits).sum()
    g = th - p @ th                               # d log p(x) / d a for p = softmax(th a)
    C = rng.uniform(0, 5, size=n)
    exact = (p * C) @ g
    mean = np.zeros(K)
    biased = np.zeros(K)
    for tup in it.product(range(n), repeat=S):
        w = np.prod(p[list(tup)])
        A = sum(C[x] * g[x] for x in tup)
        G = sum(g[x] for x in tup)
        mean += w * loo_score_gradient(A[None], G[None], np.array([C[list(tup)].sum()]), S)[0]
        cb = C[list(tup)].mean()
        biased += w * sum((C[x] - cb) * g[x] for x in tup) / S
    assert np.allclose(mean, exact, atol=1e-12)
    assert np.allclose(biased, (1 - 1 / S) * exact, atol=1e-12)


def _fake_graph_executor():
    from paper_2103_17226_amd.serve import GraphExecutor

    class G:
        info = {"n_internal": 10000, "n_qubits": 8, "n_angles": 2, "n_words": 3}

        def sample_shape(self, dtype, chains):
            return "stream", min(chains, 4096)

        def workspace_size(self, dtype, batch, op):
            return 1024 * batch
    from paper_2103_17226_amd import _lib
    ex = object.__new__(GraphExecutor)
    ex.graphs = {"g": G()}
    ex.L = _lib
    return ex


def test_graph_executor_splits_cover_the_request_exactly():
    ex = _fake_graph_executor()
    limit = 0.5
    for P, S, by_chains in ((64, 4000, False), (2, 40000, True)):
        r = Request(graph="g", theta=np.arange(P * 2, dtype=float).reshape(P, 2), samples=S, grad=True,
                    chain_offset=11)
        assert ex.cost(r) > limit
        parts = ex.split(r, limit)
        assert parts and all(ex.cost(u) <= limit for u in parts)
        assert any(u.part[4] - u.part[3] < S for u in parts) == by_chains
        covered = np.zeros((P, S), dtype=int)
        for u in parts:
            _, p0, p1, c0, c1, s0, s1 = u.part
            assert (s0, s1) == (0, r.burn_in + 1) and u.after == -1
            covered[p0:p1, c0:c1] += 1
            assert u.chain_offset == 11 + p0 * S + c0 and u.samples == c1 - c0
            assert np.array_equal(u.theta, r.theta[p0:p1])
        assert (covered == 1).all()
    # a memory cap: parts small enough for it
    big = Request(graph="g", theta=np.zeros((3, 2)), samples=9000, grad=False)
    parts = ex.split(big, float("inf"), max_bytes=2 * ex.footprint(Request(graph="g", theta=np.zeros((1, 2)),
                                                                               samples=1000)))
    assert parts and all(ex.footprint(u) <= 2 * ex.footprint(Request(graph="g", theta=np.zeros((1, 2)),
                                                                         samples=1000)) for u in parts)
    assert sum(u.samples * (u.part[2] - u.part[1]) for u in parts) == 27000
    # a limit below one chain's time: slices of the sweeps of one group of
    # concurrent chains, each resuming the slice before it, none refused
    big = Request(graph="g", theta=np.zeros((3, 2)), samples=9000, grad=True, burn_in=10)
    one = Request(graph="g", theta=np.zeros((1, 2)), samples=1, burn_in=10)
    parts = ex.split(big, ex.cost(one) / 4)
    assert parts
    assert all(ex.cost(u) <= ex.cost(one) / 4 for u in parts if not u.grad)
    sweeps = {}
    for k, u in enumerate(parts):
        _, p0, p1, c0, c1, s0, s1 = u.part
        assert p1 == p0 + 1 and u.first_sweep == s0 and u.burn_in == s1 - s0 - 1
        assert u.grad == (s1 == 11)
        chain = sweeps.setdefault((p0, c0, c1), [])
        assert u.after == (-1 if not chain else chain[-1][2])
        chain.append((s0, s1, k))
    for (p0, c0, c1), sl in sweeps.items():
        assert sl[0][0] == 0 and sl[-1][1] == 11 and all(a[1] == b[0] for a, b in zip(sl, sl[1:]))
    assert sum(c1 - c0 for p0, c0, c1 in sweeps) == 27000 and len(parts) > len(sweeps)
    # amplitudes: rows of each parameter set go to the parts that hold it
    # (whole sets while they fit, else slices of one set's rows)
    B = 40000
    for P in (7, 1):
        po = np.random.default_rng(P).integers(0, P, size=B).astype(np.int32)
        e = Request(graph="g", theta=np.arange(P * 2, dtype=float).reshape(P, 2),
                    evidence=np.arange(B * 3, dtype=np.uint64).reshape(B, 3), param_of=po,
                    weight=np.arange(B, dtype=float), grad=True)
        assert ex.cost(e) > 0.004
        parts = ex.split(e, 0.004)
        assert len(parts) > 1 and all(ex.cost(u) <= 0.004 for u in parts)
        seen = np.zeros(B, dtype=int)
        for u in parts:
            _, p0, p1, rows = u.part
            seen[rows] += 1
            assert np.array_equal(u.param_of + p0, po[rows]) and np.array_equal(u.weight, e.weight[rows])
            assert np.array_equal(u.evidence, e.evidence[rows])
        assert (seen == 1).all()


def test_parts_of_a_split_request_leave_streams_for_others():
    clock = Clock()
    ex = SplitExecutor(clock, n_streams=4)
    srv = Server(ex, mem_budget=1000, clock=clock, max_seconds=1.0, part_streams=2)
    big = srv.submit(req(10, 0.0, val=0, samples=6))          # six one-unit parts
    small = srv.submit(req(10, 0.0, val=50, samples=1))
    srv.step()
    first = [x[0] for x in ex.launched]
    assert first == [[1], [2], [7]]              # two parts (rids 1, 2), then the small request (rid 7)
    assert [r for r in srv.queue if r.parent is None] == []
    run_until_idle(srv, clock)
    assert big.result() == [float(u) for u in range(6)] and small.result() == [50.0]


def test_whole_requests_keep_their_streams_while_a_long_request_runs():
    # a request of 12 one-second units is split into twelve parts on the one
    # stream kept for parts; one-second whole requests arriving meanwhile
    # use the other stream and finish within a second or two of arriving
    clock = Clock()
    ex = SplitExecutor(clock, n_streams=2)
    srv = Server(ex, mem_budget=1000, clock=clock, max_seconds=1.0, part_streams=1, part_share=0.5)
    big = srv.submit(req(10, 0.0, val=0, samples=12))
    smalls = []
    for k in range(8):
        clock.t = float(k)
        smalls.append(srv.submit(req(10, 0.0, val=100 + k, samples=1)))
        srv.step()
        clock.t += 0.5
        srv.step()
    run_until_idle(srv, clock)
    assert big.result() == [float(u) for u in range(12)]
    assert [f.result() for f in smalls] == [[100.0 + k] for k in range(8)]
    st = srv.latency_stats()
    assert st["whole"]["completed"] == 8 and st["split"]["completed"] == 1
    assert st["whole"]["p99_ms"] <= 1500.0
    assert st["split"]["p50_ms"] >= 12000.0
    parts = [(stream, share) for is_part, stream, share in ex.kinds if is_part]
    wholes = [stream for is_part, stream, _ in ex.kinds if not is_part]
    assert len(parts) == 12 and all(share == 0.5 for _, share in parts)
    assert len(wholes) == 8 and srv.parts_inflight == 0


def test_parts_carry_their_share_and_split_requests_have_their_own_limit():
    clock = Clock()
    ex = SplitExecutor(clock, n_streams=4)
    srv = Server(ex, mem_budget=1000, clock=clock, max_seconds=2.0, max_split=2, part_share=0.25, max_queue=1)
    a = srv.submit(req(10, 0.0, val=0, samples=5))
    b = srv.submit(req(10, 0.0, val=0, samples=5))
    c = srv.submit(req(10, 0.0, val=0, samples=5))             # a third split request: refused
    w = srv.submit(req(10, 0.0, val=3, samples=1))             # the whole-request queue is not full of parts
    with pytest.raises(AdmissionError):
        c.result(timeout=0)
    assert srv.rejected_queue == 1 and len(srv.queue) == 1 and len(srv.split_queue) == 2
    assert all(u.share == 0.25 for p in srv.split_queue for u in p.part["todo"])
    run_until_idle(srv, clock)
    assert a.result() == b.result() == [float(u) for u in range(5)] and w.result() == [3.0]
    d = srv.submit(req(10, 0.0, val=0, samples=5))             # room again once they completed
    run_until_idle(srv, clock)
    assert d.result() == [float(u) for u in range(5)] and srv.split_active == 0


def test_a_split_request_is_cancelled_only_before_its_first_part():
    clock = Clock()
    ex = SplitExecutor(clock, n_streams=1)
    srv = Server(ex, mem_budget=1000, clock=clock, max_seconds=1.0)
    first = srv.submit(req(10, 0.0, val=0, samples=3))
    second = srv.submit(req(10, 0.0, val=0, samples=3))
    srv.step()                                                  # the first part of `first` launches
    assert not srv.cancel(first)
    assert srv.cancel(second) and second.cancelled()
    run_until_idle(srv, clock)
    assert first.result() == [0.0, 1.0, 2.0] and srv.split_active == 0


def test_split_requests_go_shortest_first_and_a_full_backlog_refuses_more():
    clock = Clock()
    ex = SplitExecutor(clock, n_streams=1)
    srv = Server(ex, mem_budget=1000, clock=clock, max_seconds=1.0, split_backlog=10.0)
    long_ = srv.submit(req(10, 0.0, val=0, samples=8))         # admitted: nothing was waiting
    short = srv.submit(req(10, 0.0, val=0, samples=2))         # 8 s waiting < 10 s: admitted
    more = srv.submit(req(10, 0.0, val=0, samples=3))          # 10 s waiting: refused
    with pytest.raises(AdmissionError):
        more.result(timeout=0)
    run_until_idle(srv, clock)
    assert short.result() == [0.0, 1.0] and long_.result() == [float(u) for u in range(8)]
    done = {id(r.future): r.t_done for r in srv.completed}
    assert done[id(short)] < done[id(long_)]                    # the short one did not wait for the long one
    assert srv.rejected_queue == 1
    # a lone request larger than the backlog limit is still admitted
    huge = srv.submit(req(10, 0.0, val=0, samples=30))
    run_until_idle(srv, clock, limit=5000)
    assert huge.result() == [float(u) for u in range(30)]


def test_an_old_split_request_is_not_starved_by_shorter_ones():
    # ageing: each second waited counts as one second less of work left
    clock = Clock()
    ex = SplitExecutor(clock, n_streams=1)
    srv = Server(ex, mem_budget=1000, clock=clock, max_seconds=1.0, max_split=100, split_backlog=1e9)
    old = srv.submit(req(10, 0.0, val=0, samples=6))
    shorts = []
    for k in range(40):                                         # a 2-unit request every 2 s
        clock.t = 2.0 * k
        shorts.append(srv.submit(req(10, 0.0, val=0, samples=2)))
        for _ in range(4):
            srv.step()
            clock.t += 0.5
    run_until_idle(srv, clock, limit=5000)
    t_old = next(r.t_done for r in srv.completed if r.future is old)
    assert t_old < 40.0


def test_resuming_parts_wait_for_the_part_they_resume():
    # two blocks of chains, each in two sweep slices; a slice launches only
    # after the slice whose chain states it resumes has completed
    clock = Clock()

    class SliceExecutor(SplitExecutor):
        def split(self, req, limit, max_bytes=None):
            out = []
            for k in range(4):
                u = Request(graph=req.graph, theta=req.theta, samples=1, part=(k, k + 1))
                u.after = k - 1 if k % 2 else -1
                out.append(u)
            return out
    ex = SliceExecutor(clock, n_streams=4)
    srv = Server(ex, mem_budget=1000, clock=clock, max_seconds=1.0, part_streams=2)
    f = srv.submit(req(10, 0.0, val=0, samples=4))
    run_until_idle(srv, clock, dt=0.25)
    assert f.result() == [0.0, 1.0, 2.0, 3.0]
    start = {rids[0]: t for rids, _, t in ex.launched}
    rid = sorted(start)
    assert start[rid[1]] >= start[rid[0]] + 1.0 and start[rid[3]] >= start[rid[2]] + 1.0


def test_whole_requests_go_shortest_first_with_ageing():
    clock = Clock()
    ex = FakeExecutor(clock, n_streams=1)
    srv = Server(ex, mem_budget=100, clock=clock, max_seconds=1.0)
    a = srv.submit(req(10, 0.5, val=1))
    srv.step()                                          # a holds the only stream
    b = srv.submit(req(10, 0.9, val=2))
    c = srv.submit(req(10, 0.1, val=3))
    run_until_idle(srv, clock, dt=0.05)
    order = [rids[0] for rids, _, _ in ex.launched]
    ids = {id(f): r.rid for r in srv.completed for f in [r.future]}
    assert order == [ids[id(a)], ids[id(c)], ids[id(b)]]
    # ageing: a request that has waited longer than the difference goes first
    clock.t = 100.0
    d = srv.submit(req(10, 0.5, val=4))
    srv.step()
    old = srv.submit(req(10, 0.9, val=5), t_arrive=90.0)
    new = srv.submit(req(10, 0.1, val=6))
    run_until_idle(srv, clock, dt=0.05)
    order = [rids[0] for rids, _, _ in ex.launched][3:]
    ids = {id(r.future): r.rid for r in srv.completed}
    assert order == [ids[id(d)], ids[id(old)], ids[id(new)]]
