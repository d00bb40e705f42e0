"""Request loop over resident arithmetic circuits: continuous batching,
admission by device memory, overlap on several HIP streams.

Many variational optimizers query the same compiled circuits again and again
with new parameters and new outcomes (Sec. 3.2: compile once, query many
times): amplitude queries (upward pass), gradients (downward pass, Sec. 3.3.2)
and samples (Gibbs, Sec. 3.3.2).  The server keeps every registered AC
resident on the device and a scheduler thread that, on every tick,

  1. completes the launches that have finished (their HIP event has fired):
     results go to the request futures, and their memory and stream are
     released at once;
  2. admits queued requests in arrival order while their device-memory
     footprint (inputs, outputs, workspace) fits the budget and a stream is
     free; the head of the queue is never overtaken for memory, so a large
     request cannot starve (requests of a busy session keep their place
     while later requests go ahead);
  3. merges an admitted amplitude request with later queued ones of the same
     graph, dtype and kind into one launch.  Parameter sets are stacked and
     every element keeps its own parameter row, so each request gets what it
     would get alone: the upward pass is elementwise, and gradient segments
     start on a 256-element boundary so that the fixed-order reduction adds
     the same terms in the same order (padding rows carry weight 0 and a
     parameter row of their own that is dropped).  Sampling requests run
     alone: their chains are numbered from the request's chain offset, which
     is what makes them reproducible from the seed.  A sampling request of a
     session resumes the chains that session left on the device; requests of
     one session run one at a time, in arrival order, and the chain states
     count against the memory budget until the session is closed.

Requests that arrive while others are on the device therefore start as soon
as a stream and memory free up, and their kernels overlap on the device.
A request estimated (with ``max_seconds``) to occupy the device longer than
that, or larger than the memory budget, is split into parts that each fit
-- by parameter sets, or by chains (sampling) or evidence rows (amplitudes)
of one parameter set -- and joins a second queue: its parts launch in order
on streams kept for parts (``part_streams``), each on a share of the device
(``part_share``: the executor gives the launch a workspace for that share of
the workgroups the device holds), so long requests make steady progress
while short ones keep the rest of the device.  Its result is assembled when
the last part completes and equals the unsplit request's (sampling parts
number their chains from the request's chain offset, so they draw the same
chains).  Submissions beyond ``max_queue`` waiting requests, or
``max_split`` split requests, are rejected at once, and so are requests that
cannot fit the budget even when split.  Resident session chains that leave no
room for the next launch, with nothing else on the device, are released
oldest first; a request that cannot fit even then fails.

The device work is done by an executor (``GraphExecutor`` for libqkc); the
scheduler only sees its footprint / launch / done / results calls, so tests
drive admission, merging, cancellation and failures from the host with an
executor and clock of their own.
"""
from __future__ import annotations

import collections
import itertools
import threading
import time
from concurrent.futures import Future
from dataclasses import dataclass, field
from typing import Any, Callable, Dict, List, Optional

import numpy as np

GRAD_ALIGN = 256      # elements per block of the gradient reduction


@dataclass(eq=False)
class Request:
    """One query.  ``samples == 0``: amplitudes of ``evidence`` rows (uint64
    [B, W] evidence words, row b under parameter set ``param_of[b]``), plus,
    if ``grad``, the gradient of sum_b weight[b] |f_b|^2 in theta.
    ``samples > 0``: that many Gibbs chains per parameter set, one sample per
    chain after ``burn_in`` sweeps, with the MaxCut cost of every sample, plus,
    if ``grad``, the score-function estimate of d<C>/dtheta from them.
    A sampling request with a ``session`` resumes that session's chains on the
    graph (kept on the device since its previous request) when P and S match,
    so consecutive optimiser iterations need little burn-in."""
    graph: str
    theta: np.ndarray                        # float64 [P, K]
    evidence: Optional[np.ndarray] = None    # uint64 [B, W]
    param_of: Optional[np.ndarray] = None    # int32 [B]
    weight: Optional[np.ndarray] = None      # float64 [B] (grad of an eval request)
    samples: int = 0
    grad: bool = False
    burn_in: int = 10
    seed: int = 1
    dtype: str = "c64"
    session: Optional[str] = None
    chain_offset: int = 0                    # RNG number of the first chain (parts of a split request)
    share: float = 1.0                       # fraction of the device a launch may hold (parts: less)
    est: float = 0.0                         # estimated device seconds (set by the server)
    first_sweep: int = 0                     # sweep number of the first sweep (a part resuming chains)
    after: int = -1                          # index of the part whose chains this part resumes
    # filled in by the server
    rid: int = -1
    t_arrive: float = 0.0
    t_start: float = 0.0
    t_launched: float = 0.0
    t_done: float = 0.0
    footprint: int = 0
    future: Future = field(default_factory=Future, repr=False)
    parent: Any = field(default=None, repr=False)    # the split request this part belongs to
    part: Any = field(default=None, repr=False)      # the executor's description of the part

    @property
    def kind(self) -> str:
        return "sample" if self.samples > 0 else "eval"

    @property
    def n_params(self) -> int:
        return int(np.asarray(self.theta).reshape(-1, np.asarray(self.theta).shape[-1]).shape[0])

    @property
    def n_rows(self) -> int:
        return 0 if self.evidence is None else int(self.evidence.shape[0])


class AdmissionError(RuntimeError):
    """The request can never fit, or the queue is full."""


class Server:
    """Continuous-batching scheduler over an executor.

    The executor provides ``n_streams``, ``footprint(req) -> bytes``,
    ``can_merge(a, b) -> bool``, ``launch(batch, stream) -> handle``,
    ``done(handle) -> bool`` and ``results(handle) -> list`` (one result per
    request of the batch, in order), and ``cost(req) -> estimated device
    seconds`` and ``split(req, limit, max_bytes)`` if ``max_seconds`` is used.
    ``launch``, ``done`` and ``results`` may raise; the requests of that batch
    then fail with the exception.  With ``request_timeout`` a launch still
    running that long after it started fails its requests with TimeoutError
    at once; its memory and stream return when the device finishes.

    Split requests form a second class: at most ``max_split`` of them wait or
    run at once, and one more is admitted only if the estimated device time
    of the parts still waiting, with its own, stays within ``split_backlog``
    seconds, or if no part is waiting (a request is never refused for its
    own size alone).  Their parts hold at most
    ``part_streams`` streams in total (kept free for them while parts wait);
    the next part comes from the split request with the least estimated work
    left, less the seconds it has waited; and each part runs on
    ``part_share`` of the device (``Request.share``, for the executor), so
    whole requests keep the rest of the device while long ones progress."""

    def __init__(self, executor, mem_budget: int, clock: Callable[[], float] = time.perf_counter,
                 max_queue: int = 1 << 30, max_merge: int = 64, max_seconds: Optional[float] = None,
                 request_timeout: Optional[float] = None, tick: float = 1e-4, part_streams: int = 1,
                 part_share: float = 0.5, max_split: int = 4, split_backlog: float = 30.0):
        if mem_budget <= 0:
            raise ValueError("mem_budget must be positive")
        if not 0.0 < part_share <= 1.0:
            raise ValueError("part_share must be in (0, 1]")
        self.ex = executor
        self.budget = int(mem_budget)
        self.clock = clock
        self.max_queue = int(max_queue)
        self.max_merge = max(1, int(max_merge))
        self.max_seconds = max_seconds
        self.request_timeout = request_timeout
        self.tick = tick
        self.part_streams = max(1, min(int(part_streams), executor.n_streams))
        self.part_share = float(part_share)
        self.max_split = max(1, int(max_split))
        self.split_backlog = float(split_backlog)
        self.queue: collections.deque = collections.deque()        # whole requests, arrival order
        self.split_queue: collections.deque = collections.deque()  # split requests with parts to launch
        self.split_active = 0                       # split requests not yet completed or failed
        self.parts_inflight = 0
        self.inflight: List[tuple] = []            # (handle, [requests], stream, bytes)
        self.free_streams = list(range(executor.n_streams))
        self.used = 0
        self.peak_used = 0
        self.lock = threading.Lock()
        self._stop = threading.Event()
        self.thread: Optional[threading.Thread] = None
        self._ids = itertools.count()
        self.completed: List[Request] = []
        self.failed = 0
        self.rejected_memory = 0
        self.rejected_queue = 0
        self.rejected_cost = 0
        self.rejected_invalid = 0
        self.split_requests = 0
        self.split_parts = 0
        self.evicted_sessions = 0
        self.timed_out = 0
        self.cancelled = 0
        self.launches = 0
        self.merged = 0
        self.max_inflight = 0
        self.busy_sessions = set()
        self.launching = 0                          # batches taken from the queue, not yet in flight

    # ------------------------------------------------------------------ API
    def submit(self, req: Request, t_arrive: Optional[float] = None) -> Future:
        """Queue a request; ``t_arrive`` (default: now) is when it arrived,
        for callers that replay a schedule of arrivals.  A request that
        cannot be admitted is refused at once, before any splitting work."""
        req.rid = next(self._ids)
        req.t_arrive = self.clock() if t_arrive is None else float(t_arrive)
        if req.kind == "sample" and req.grad and req.samples < 2:
            return self._refuse(req, "invalid", "a sampled gradient needs at least 2 samples per parameter set "
                                                "(leave-one-out baseline)")
        req.est = float(self.ex.cost(req)) if self.max_seconds is not None else 0.0
        over_time = self.max_seconds is not None and req.est > self.max_seconds
        over_memory = False
        if not over_time:
            req.footprint = int(self.ex.footprint(req))
            over_memory = req.footprint > self.budget
        if not (over_time or over_memory):
            with self.lock:
                if len(self.queue) >= self.max_queue:
                    return self._refuse(req, "queue", f"queue full ({self.max_queue} waiting)")
                self.queue.append(req)
            return req.future
        if not hasattr(self.ex, "split") or req.session is not None:
            if over_memory:
                return self._refuse(req, "memory", f"request needs {req.footprint} bytes of device memory, "
                                                   f"the budget is {self.budget}")
            return self._refuse(req, "cost", f"request would hold the device ~{float(self.ex.cost(req)):.3g} s, "
                                             f"the limit is {self.max_seconds:.3g} s, and it cannot be split")
        with self.lock:
            full = self._split_full(req.est)
        if full:
            return self._refuse(req, "queue", f"split queue full: {full}")
        limit = self.max_seconds if self.max_seconds is not None else float("inf")
        parts = self.ex.split(req, limit, max_bytes=self.budget)
        if not parts:
            if over_memory:
                return self._refuse(req, "memory", f"request needs {req.footprint} bytes of device memory, "
                                                   f"the budget is {self.budget}, and it cannot be split")
            return self._refuse(req, "cost", f"request would hold the device ~{float(self.ex.cost(req)):.3g} s, "
                                             f"the limit is {self.max_seconds:.3g} s, and it cannot be split")
        costs = []
        for u in parts:
            u.share = self.part_share
            u.footprint = int(self.ex.footprint(u))
            if u.footprint > self.budget:
                return self._refuse(req, "memory", f"a part needs {u.footprint} bytes of device memory, "
                                                   f"the budget is {self.budget}")
            costs.append(float(self.ex.cost(u)) if self.max_seconds is not None else 0.0)
        with self.lock:
            full = self._split_full(sum(costs))
            if full:
                return self._refuse(req, "queue", f"split queue full: {full}")
            req.part = {"n": len(parts), "done": 0, "outs": [None] * len(parts), "failed": False,
                        "descs": [u.part for u in parts], "inflight": 0,
                        "todo": collections.deque(parts), "costs": collections.deque(costs)}
            for k, u in enumerate(parts):
                u.rid = next(self._ids)
                u.t_arrive = req.t_arrive
                u.parent = req
                u.part = (k, u.part)
            self.split_requests += 1
            self.split_parts += len(parts)
            self.split_active += 1
            self.split_queue.append(req)
        return req.future

    def _split_full(self, est: float) -> str:
        """Why a split request of ``est`` estimated seconds cannot be
        admitted now ("" if it can): the split class holds ``max_split``
        requests, or its waiting parts and this one would exceed
        ``split_backlog`` seconds -- unless nothing is waiting, so a request
        is never refused for its own size alone.  Called with the lock held."""
        if self.split_active >= self.max_split:
            return f"{self.split_active} split requests"
        backlog = self._split_backlog()
        if backlog > 0.0 and backlog + est > self.split_backlog:
            return f"~{backlog:.3g} s of parts waiting"
        return ""

    def _refuse(self, req: Request, why: str, msg: str) -> Future:
        setattr(self, "rejected_" + why, getattr(self, "rejected_" + why) + 1)
        req.future.set_exception(AdmissionError(msg))
        return req.future

    def cancel(self, fut: Future) -> bool:
        """Cancel a request that is still waiting (a split request only
        before its first part launched); one already on the device runs to
        completion (returns False)."""
        with self.lock:
            for r in self.queue:
                if r.future is fut:
                    self.queue.remove(r)
                    break
            else:
                par = next((r for r in self.split_queue if r.future is fut), None)
                if par is None or len(par.part["todo"]) != par.part["n"]:
                    return False
                self.split_queue.remove(par)
                self.split_active -= 1
            self.cancelled += 1
            fut.cancel()
            return True

    def start(self):
        if self.thread is not None:
            raise RuntimeError("server already started")
        self._stop.clear()
        self.thread = threading.Thread(target=self._run, name="ac-serve", daemon=True)
        self.thread.start()

    def idle(self) -> bool:
        with self.lock:
            return not self.queue and not self.split_queue and not self.inflight and not self.launching

    def stop(self, drain: bool = True, timeout: float = 600.0):
        """Stop the scheduler thread, after the queue and the device drain if
        ``drain``; waiting requests left behind are cancelled."""
        if drain and self.thread is not None:
            t0 = time.perf_counter()
            while not self.idle() and time.perf_counter() - t0 < timeout:
                time.sleep(self.tick)
        self._stop.set()
        if self.thread is not None:
            self.thread.join(timeout)
            self.thread = None
        # with drain, launches still on the device complete here (the thread has exited)
        t0 = time.perf_counter()
        while drain and self.inflight and time.perf_counter() - t0 < timeout:
            if not self._complete():
                time.sleep(self.tick)
        with self.lock:
            left = list(self.queue) + list(self.split_queue)
            self.queue.clear()
            self.split_queue.clear()
            for r in left:
                if not r.future.done():
                    self.cancelled += 1
                    r.future.cancel()

    # ------------------------------------------------------------ scheduler
    def _fail(self, reqs, exc):
        for r in reqs:
            r.t_done = self.clock()
            if r.parent is not None:                 # a part: the split request fails once
                r.future.set_exception(exc)
                par = r.parent
                if not par.part["failed"]:
                    par.part["failed"] = True
                    par.t_done = r.t_done
                    self.failed += 1
                    with self.lock:
                        self.split_active -= 1
                        par.part["todo"].clear()
                        par.part["costs"].clear()
                        if par in self.split_queue:
                            self.split_queue.remove(par)
                    if hasattr(self.ex, "discard"):
                        self.ex.discard(par)
                    if not par.future.done():
                        par.future.set_exception(exc)
                continue
            self.failed += 1
            if not r.future.done():
                r.future.set_exception(exc)

    def _finish(self, r, out, now):
        """A request or a part completed with the executor's output."""
        r.t_done = now
        if r.parent is None:
            self.completed.append(r)
            r.future.set_result(self.ex.finalize(r, out) if hasattr(self.ex, "finalize") else out)
            return 1
        r.future.set_result(out)
        par, st = r.parent, r.parent.part
        st["outs"][r.part[0]] = out
        st["done"] += 1
        if st["done"] < st["n"] or st["failed"] or par.future.done():
            return 0
        par.t_done = now
        with self.lock:
            self.split_active -= 1
        try:
            res = self.ex.combine(par, st["outs"])
        except Exception as exc:
            self.failed += 1
            par.future.set_exception(exc)
            return 0
        self.completed.append(par)
        par.future.set_result(res)
        return 1

    def _complete(self) -> int:
        finished = 0
        still = []
        for h, reqs, stream, nbytes in self.inflight:
            try:
                ready = self.ex.done(h)
            except Exception as exc:           # device error: fail the batch
                ready, outs = True, exc
            else:
                outs = None
                if ready:
                    try:
                        outs = self.ex.results(h)
                    except Exception as exc:
                        outs = exc
            if not ready:
                if self.request_timeout is not None and self.clock() - reqs[0].t_launched > self.request_timeout:
                    # the kernels cannot be stopped: the callers get an error now and
                    # the memory and stream are released when the launch completes
                    pending = [r for r in reqs if not r.future.done()]
                    if pending:
                        self.timed_out += len(pending)
                        self._fail(pending, TimeoutError(
                            f"request still on the device after {self.request_timeout:.3g} s"))
                still.append((h, reqs, stream, nbytes))
                continue
            if isinstance(outs, Exception):
                self._fail([r for r in reqs if not r.future.done()], outs)
            else:
                now = self.clock()
                for r, o in zip(reqs, outs):
                    if r.future.done():            # timed out earlier
                        continue
                    finished += self._finish(r, o, now)
            with self.lock:
                self.used -= nbytes
                self.free_streams.append(stream)
                self._release(reqs)
        self.inflight = still
        return finished

    def _release(self, reqs):
        for r in reqs:
            if r.session is not None:
                self.busy_sessions.discard((r.graph, r.session))
            if r.parent is not None:
                r.parent.part["inflight"] -= 1
                self.parts_inflight -= 1

    def _make_room(self, need: int, resident: int) -> int:
        """Nothing is on the device and ``need`` bytes do not fit next to
        the resident session chains: release idle ones, least recently used
        first; returns the resident bytes left."""
        if hasattr(self.ex, "evict_sessions"):
            self.evicted_sessions += self.ex.evict_sessions(resident + need - self.budget, self.busy_sessions)
            resident = self.ex.resident_bytes()
        return resident

    def _split_backlog(self) -> float:
        """Estimated device seconds of the parts still waiting."""
        return sum(sum(p.part["costs"]) for p in self.split_queue if not p.part["failed"])

    @staticmethod
    def _part_ready(par) -> bool:
        """The next part of a split request can launch: the part whose
        chains it resumes, if any, has completed."""
        u = par.part["todo"][0]
        return u.after < 0 or par.part["outs"][u.after] is not None

    def _next_split(self):
        """The split request whose parts go next, among those whose next
        part is ready: least estimated work left, less the seconds it has
        waited (shortest first, with ageing); None if none is ready."""
        now = self.clock()
        ready = [p for p in self.split_queue if self._part_ready(p)]
        if not ready:
            return None
        return min(ready, key=lambda p: (sum(p.part["costs"]) - (now - p.t_arrive), p.rid))

    def _take_part(self, resident: int):
        """The next part of a split request (``_next_split``), if a stream
        for parts and its memory are free; called with the lock held."""
        while self.split_queue and self.parts_inflight < self.part_streams and self.free_streams:
            for p in [p for p in self.split_queue if p.part["failed"] or not p.part["todo"]]:
                self.split_queue.remove(p)
            if not self.split_queue:
                break
            par = self._next_split()
            if par is None:
                return None
            st = par.part
            u = st["todo"][0]
            if self.used + resident + u.footprint > self.budget:
                if self.used or self.inflight or self.launching:
                    return None                    # room comes back as launches complete
                resident = self._make_room(u.footprint, resident)
                if resident + u.footprint > self.budget:
                    self.split_queue.remove(par)
                    st["todo"].clear()
                    st["costs"].clear()
                    st["failed"] = True
                    self.split_active -= 1
                    self.rejected_memory += 1
                    if hasattr(self.ex, "discard"):
                        self.ex.discard(par)
                    if not par.future.done():
                        par.future.set_exception(AdmissionError(
                            f"part needs {u.footprint} bytes next to {resident} bytes of resident session "
                            f"chains in use, the budget is {self.budget}"))
                    continue
            st["todo"].popleft()
            st["costs"].popleft()
            if not st["todo"]:
                self.split_queue.remove(par)
            st["inflight"] += 1
            self.parts_inflight += 1
            self.launching += 1
            stream = self.free_streams.pop(0)
            self.used += u.footprint
            self.peak_used = max(self.peak_used, self.used)
            return [u], stream, u.footprint
        return None

    def _take_batch(self):
        """Pop the next launch if it fits; called with the lock held.  Parts
        of split requests go first on the streams kept for them.  Of the
        whole requests whose session is idle (requests of a busy session
        keep their place), the one with the least estimated device time less
        the seconds it has waited leads -- shortest first, with ageing; in
        arrival order without ``max_seconds`` -- and no other request
        overtakes it for memory."""
        if not self.free_streams:
            return None
        resident = self.ex.resident_bytes() if hasattr(self.ex, "resident_bytes") else 0
        got = self._take_part(resident)
        if got is not None:
            return got
        waiting_parts = any(not p.part["failed"] and p.part["todo"] and self._part_ready(p) for p in self.split_queue)
        keep_free = max(0, self.part_streams - self.parts_inflight) if waiting_parts else 0
        if not self.queue or len(self.free_streams) <= keep_free:
            return None
        now = self.clock()
        ready = [(r.est - (now - r.t_arrive), r.rid, k) for k, r in enumerate(self.queue)
                 if not (r.session is not None and (r.graph, r.session) in self.busy_sessions)]
        if not ready:
            return None
        idx = min(ready)[2]
        head = self.queue[idx]
        if self.used + resident + head.footprint > self.budget:
            if self.used or self.inflight or self.launching:
                return None                        # room comes back as launches complete
            resident = self._make_room(head.footprint, resident)
            if resident + head.footprint > self.budget:
                del self.queue[idx]
                self.rejected_memory += 1
                if not head.future.done():
                    head.future.set_exception(AdmissionError(
                        f"request needs {head.footprint} bytes next to {resident} bytes of resident session "
                        f"chains in use, the budget is {self.budget}"))
                return self._take_batch()
        del self.queue[idx]
        batch, total = [head], head.footprint
        if head.kind == "eval" and self.max_merge > 1:
            keep = collections.deque()
            while self.queue and len(batch) < self.max_merge:
                r = self.queue.popleft()
                if self.ex.can_merge(head, r) and self.used + resident + total + r.footprint <= self.budget:
                    batch.append(r)
                    total += r.footprint
                else:
                    keep.append(r)
            keep.extend(self.queue)
            self.queue = keep
        if head.session is not None:
            self.busy_sessions.add((head.graph, head.session))
        self.launching += 1
        stream = self.free_streams.pop(0)
        self.used += total
        self.peak_used = max(self.peak_used, self.used)
        return batch, stream, total

    def close_session(self, graph: str, session: str):
        """Drop a session's resident chains (after its requests complete)."""
        if hasattr(self.ex, "drop_session"):
            self.ex.drop_session(graph, session)

    def step(self) -> int:
        """One scheduler tick; returns the number of requests completed."""
        finished = self._complete()
        while True:
            with self.lock:
                got = self._take_batch()
            if got is None:
                break
            batch, stream, total = got
            now = self.clock()
            for r in batch:
                r.t_start = now
                if r.parent is not None and not r.parent.t_start:
                    r.parent.t_start = now
            try:
                handle = self.ex.launch(batch, stream)
            except Exception as exc:
                self._fail(batch, exc)
                with self.lock:
                    self.used -= total
                    self.free_streams.append(stream)
                    self._release(batch)
                    self.launching -= 1
                continue
            now = self.clock()
            for r in batch:
                r.t_launched = now
                if r.parent is not None and not r.parent.t_launched:
                    r.parent.t_launched = now
            self.launches += 1
            self.merged += len(batch) - 1
            with self.lock:
                self.inflight.append((handle, batch, stream, total))
                self.launching -= 1
            self.max_inflight = max(self.max_inflight, len(self.inflight))
        return finished

    def _run(self):
        while not self._stop.is_set():
            if not self.step():
                time.sleep(self.tick)

    # --------------------------------------------------------------- stats
    @staticmethod
    def _lat(done) -> Dict[str, Any]:
        lat = np.array([r.t_done - r.t_arrive for r in done])
        if not len(lat):
            return {"completed": 0}
        return {"completed": len(done), "p50_ms": float(np.percentile(lat, 50) * 1e3),
                "p99_ms": float(np.percentile(lat, 99) * 1e3), "mean_ms": float(lat.mean() * 1e3)}

    def latency_stats(self, since: float = float("-inf")) -> Dict[str, Any]:
        """Latency (arrival to completion) over requests that arrived at or
        after ``since``, with counts of every outcome; ``whole`` and
        ``split`` give the latency of the two classes apart."""
        done = [r for r in self.completed if r.t_arrive >= since]
        out: Dict[str, Any] = {"completed": len(done), "failed": self.failed,
                               "rejected_memory": self.rejected_memory,
                               "rejected_queue": self.rejected_queue, "rejected_cost": self.rejected_cost,
                               "rejected_invalid": self.rejected_invalid, "timed_out": self.timed_out,
                               "split_requests": self.split_requests, "split_parts": self.split_parts,
                               "evicted_sessions": self.evicted_sessions,
                               "cancelled": self.cancelled,
                               "launches": self.launches, "merged": self.merged,
                               "max_inflight": self.max_inflight, "peak_bytes": self.peak_used}
        allst = self._lat(done)
        if allst["completed"]:
            out.update(p50_ms=allst["p50_ms"], p99_ms=allst["p99_ms"], mean_ms=allst["mean_ms"])
        out["whole"] = self._lat([r for r in done if not isinstance(r.part, dict)])
        out["split"] = self._lat([r for r in done if isinstance(r.part, dict)])
        return out


def loo_score_gradient(A, G, cost_sum, S: int):
    """Score-function estimate of d<C>/dtheta per parameter set from S
    samples s_i with the leave-one-out baseline,
        (1/S) sum_i (C_i - (sum_j C_j - C_i)/(S - 1)) g_i
      = (A - (sum_j C_j / S) G) / (S - 1),
    with g_i = d log |f(s_i)|^2 / d theta, A = sum_i C_i g_i (rows [P, K]),
    G = sum_i g_i and cost_sum = sum_i C_i [P].  Each sample's baseline is
    independent of it, so the estimate is unbiased (S >= 2)."""
    A = np.asarray(A, dtype=np.float64)
    G = np.asarray(G, dtype=np.float64)
    cbar = np.asarray(cost_sum, dtype=np.float64).reshape(-1, 1) / float(S)
    return (A - cbar * G) / float(S - 1)


def padded_rows(n_rows: int, grad: bool) -> int:
    """Rows a request occupies in a merged launch: gradient segments are
    rounded up to a whole reduction block."""
    return -(-n_rows // GRAD_ALIGN) * GRAD_ALIGN if grad else n_rows


def stack_eval_batch(batch: List[Request], K: int, W: int, grad: bool):
    """Stack the amplitude requests of one launch.

    Returns (theta [P_all, K], evidence [B_all, W] uint64, param_of [B_all],
    weight [B_all] or None, spans) with spans[i] = (p0, P, b0, B): request i's
    parameter rows and evidence rows.  With ``grad`` every request's rows
    start on a multiple of GRAD_ALIGN and the rows that pad it carry weight 0
    and point at one extra all-zero parameter row (the last) whose gradient
    is dropped."""
    thetas, evs, pos, wts, spans = [], [], [], [], []
    p0 = b0 = 0
    for r in batch:
        P, B = r.n_params, r.n_rows
        th = np.asarray(r.theta, dtype=np.float64).reshape(P, K)
        po = np.zeros(B, dtype=np.int32) if r.param_of is None else np.asarray(r.param_of, dtype=np.int32)
        if po.shape != (B,):
            raise ValueError("param_of must have one entry per evidence row")
        if B and (po.min() < 0 or po.max() >= P):
            raise ValueError("param_of entries must lie in [0, P)")
        ev = np.asarray(r.evidence, dtype=np.uint64).reshape(B, W)
        thetas.append(th)
        evs.append(ev)
        pos.append(po + p0)
        if grad:
            w = np.ones(B) if r.weight is None else np.asarray(r.weight, dtype=np.float64).reshape(B)
            wts.append(w)
        spans.append((p0, P, b0, B))
        p0 += P
        b0 += B
        pad = padded_rows(B, grad) - B
        if pad:
            evs.append(np.zeros((pad, W), dtype=np.uint64))
            pos.append(np.full(pad, -1, dtype=np.int32))
            wts.append(np.zeros(pad))
            b0 += pad
    if grad:
        thetas.append(np.zeros((1, K)))
    theta = np.concatenate(thetas) if thetas else np.zeros((0, K))
    po = np.concatenate(pos) if pos else np.zeros(0, dtype=np.int32)
    po[po < 0] = theta.shape[0] - 1
    ev = np.concatenate(evs) if evs else np.zeros((0, W), dtype=np.uint64)
    wt = (np.concatenate(wts) if wts else np.zeros(0)) if grad else None
    return theta, ev, po, wt, spans


# ---------------------------------------------------------------------------
# executor over libqkc graphs
# ---------------------------------------------------------------------------

class GraphExecutor:
    """Runs requests on resident ``ACGraph`` objects, one HIP stream per slot.

    Inputs are staged through pinned host memory and copied on the request's
    stream; results are copied back on the same stream into pinned host
    buffers before the completion event, so the scheduler never blocks on the
    device.  Every launch brings its own workspace (the graph's cached one is
    shared, and launches of one graph overlap).

    HIP maps streams onto the process's hardware queues (GPU_MAX_HW_QUEUES,
    read when HIP starts; 4 unless set), and launches on streams that share a
    queue run one after the other: with fewer queues than streams a short
    request can wait behind a long kernel of another stream.  Give the
    process at least one queue per stream."""

    def __init__(self, graphs: Dict[str, Any], cost_edges: Optional[Dict[str, Any]] = None,
                 n_streams: int = 8, device: int = 0):
        import torch
        from . import _lib
        self.torch = torch
        self.L = _lib
        self.graphs = graphs
        self.n_streams = int(n_streams)
        self.device = torch.device("cuda", device)
        self.streams = [torch.cuda.Stream(device=self.device) for _ in range(self.n_streams)]
        self.sessions = {}        # (graph, session) -> [states [P*S, W] int64 on device, next sweep, P, S, last use]
        self._carry = {}          # (split request id, p0, c0) -> chain states between slices of its sweeps
        self._sess_lock = threading.Lock()
        self._uses = itertools.count()
        self.edges = {}
        for name, e in (cost_edges or {}).items():
            self.edges[name] = torch.as_tensor(np.asarray(e, dtype=np.int32).reshape(-1, 2)).to(self.device)

    # ---------------------------------------------------------- sizing
    def can_merge(self, a: Request, b: Request) -> bool:
        return (a.kind == "eval" and b.kind == "eval" and a.graph == b.graph and a.dtype == b.dtype
                and a.grad == b.grad)

    def footprint(self, req: Request) -> int:
        """Device bytes of one request: workspace, inputs and outputs."""
        L = self.L
        g = self.graphs[req.graph]
        info = g.info
        cs = 8 if req.dtype == "c64" else 16
        P, K, W = req.n_params, info["n_angles"], info["n_words"]
        if req.kind == "sample":
            chains = P * int(req.samples)
            ws = self.ws_bytes(g, req.dtype, chains, L.AC_OP_SAMPLE, req.share)
            nwq = (info["n_qubits"] + 63) // 64
            io = chains * 8 * (nwq + 1) + P * K * 8
            if req.grad:
                ws = max(ws, self.ws_bytes(g, req.dtype, chains, L.AC_OP_GRAD, req.share))
                io += chains * (8 * W + 4 + 8 + cs) + P * K * 8
            return ws + io
        B = padded_rows(req.n_rows, req.grad)
        op = L.AC_OP_GRAD if req.grad else L.AC_OP_EVAL
        ws = self.ws_bytes(g, req.dtype, B, op, req.share)
        return ws + B * (8 * W + 4 + 8 + cs) + (P + 1) * K * 16

    @staticmethod
    def ws_bytes(g, dtype: str, batch: int, op: int, share: float) -> int:
        """Workspace of a launch that may hold ``share`` of the device."""
        if share >= 1.0:
            return max(g.workspace_size(dtype, batch, op), 256)
        return max(g.workspace_size_share(dtype, batch, op, share), 256)

    # device-time model for admission: a lone tile of 64 elements walks the DAG
    # level by level (latency per node step, with the 8- or 16-wave
    # workgroups the library gives small batches), a full chip streams node
    # steps at a measured rate; a request takes the larger of the two
    NODE_STEP_LATENCY = {"stream": 7.0e-8, "global": 3.0e-7, "lds": 1.0e-8, "eval": 1.0e-7}
    NODE_STEP_RATE = {"sample": 1.7e11, "eval": 1.7e11}

    def cost(self, req: Request) -> float:
        """Estimated device seconds of a request (for ``max_seconds``).
        Sampling: about n/2 + 1 rounds per sweep (a round ends at the first
        change) of three passes (up, down, leaves) over the DAG per chain, at
        the per-step latency of the kernel the library picks for this many
        chains, once per group of chains it runs at once, or at the chip's
        node-step rate when that is slower; amplitudes: one pass per row,
        three with a gradient.  A launch on a share of the device runs
        proportionally fewer chains or rows at once."""
        g = self.graphs[req.graph]
        info = g.info
        N = float(info["n_internal"])
        share = min(1.0, float(req.share))
        if req.kind == "sample":
            chains = req.n_params * int(req.samples)
            steps = 3.0 * N * (req.burn_in + 1) * (info["n_qubits"] // 2 + 1)
            if req.grad:
                steps += 3.0 * N
            kind, conc = g.sample_shape(req.dtype, chains)
            groups = -(-chains // max(int(conc * share), 1))
            lat = groups * steps * self.NODE_STEP_LATENCY[kind]
            return max(lat, chains * steps / (self.NODE_STEP_RATE["sample"] * share))
        passes = 3.0 if req.grad else 1.0
        lat = passes * N * self.NODE_STEP_LATENCY["eval"]
        return max(lat, req.n_rows * passes * N / (self.NODE_STEP_RATE["eval"] * share))

    def resident_bytes(self) -> int:
        """Device bytes of the resident session chains."""
        with self._sess_lock:
            return sum(int(v[0].numel()) * 8 for v in self.sessions.values())

    def drop_session(self, graph: str, session: str):
        with self._sess_lock:
            self.sessions.pop((graph, session), None)

    def evict_sessions(self, need: int, busy) -> int:
        """Release idle sessions' chains, least recently used first, until
        ``need`` bytes are free or none is left; returns how many."""
        n = 0
        with self._sess_lock:
            idle = sorted((v[4], k) for k, v in self.sessions.items() if k not in busy)
            for _, k in idle:
                if need <= 0:
                    break
                need -= int(self.sessions.pop(k)[0].numel()) * 8
                n += 1
        return n

    # ---------------------------------------------------------- splitting
    @staticmethod
    def _largest(fits, hi: int) -> int:
        """Largest k in [1, hi] with fits(k) (fits is monotone), else 0."""
        if hi < 1 or not fits(1):
            return 0
        lo = 1
        while lo < hi:
            mid = (lo + hi + 1) // 2
            if fits(mid):
                lo = mid
            else:
                hi = mid - 1
        return lo

    def split(self, req: Request, limit: float, max_bytes: Optional[int] = None):
        """Parts of a request whose device time would exceed ``limit``: whole
        parameter sets per part while they fit, else slices of one set's
        chains (sampling) or evidence rows (amplitudes), else (sampling)
        slices of the sweeps of a group of chains, each part resuming the
        chains of the part before it (``after``).  When one unit alone -- one
        sweep of one chain, one evidence row -- is over the limit (a large
        circuit), the limit becomes that unit's time, so a part holds what
        the device runs in that time anyway rather than being refused.  With
        ``max_bytes`` a part's device footprint stays within it too.  None if
        no part fits."""
        cap = float("inf") if max_bytes is None else max_bytes

        def ok(u, lim):
            return self.cost(u) <= lim and self.footprint(u) <= cap
        P = req.n_params
        th = np.asarray(req.theta, dtype=np.float64).reshape(P, -1)
        parts = []
        if req.kind == "sample":
            S = int(req.samples)
            sweeps = int(req.burn_in) + 1

            def part(p0, p1, c0, c1, s0=0, s1=sweeps):
                return Request(graph=req.graph, theta=th[p0:p1], samples=c1 - c0, grad=req.grad and s1 == sweeps,
                               burn_in=s1 - s0 - 1, seed=req.seed, dtype=req.dtype, first_sweep=s0,
                               chain_offset=req.chain_offset + p0 * S + c0,
                               part=("sample", p0, p1, c0, c1, s0, s1))
            limit = max(limit, self.cost(part(0, 1, 0, 1, 0, 1)) * (1.0 + 1e-9))
            pc = self._largest(lambda k: ok(part(0, k, 0, S), limit), P)
            if pc:
                return [part(p0, min(P, p0 + pc), 0, S) for p0 in range(0, P, pc)]
            sc = self._largest(lambda k: ok(part(0, 1, 0, k), limit), S)
            if sc:
                return [part(p, p + 1, c0, min(S, c0 + sc)) for p in range(P) for c0 in range(0, S, sc)]
            # one group of chains runs longer than the limit (a large circuit):
            # its sweeps in slices, each resuming the chains where the slice
            # before it left them (the same chains as one call)
            cb = self._largest(lambda k: ok(part(0, 1, 0, k, 0, 1), limit), S)
            if not cb:
                return None
            ns = max(1, self._largest(lambda k: ok(part(0, 1, 0, cb, 0, k), limit), sweeps))
            for p in range(P):
                for c0 in range(0, S, cb):
                    prev = -1
                    for s0 in range(0, sweeps, ns):
                        u = part(p, p + 1, c0, min(S, c0 + cb), s0, min(sweeps, s0 + ns))
                        u.after = prev
                        prev = len(parts)
                        parts.append(u)
            return parts
        po = np.zeros(req.n_rows, dtype=np.int64) if req.param_of is None else np.asarray(req.param_of, np.int64)
        ev = np.asarray(req.evidence, dtype=np.uint64)
        wt = None if req.weight is None else np.asarray(req.weight, dtype=np.float64)
        order = np.argsort(po, kind="stable")
        starts = np.searchsorted(po[order], np.arange(P + 1))

        def part(p0, p1, rows):
            return Request(graph=req.graph, theta=th[p0:p1], evidence=ev[rows],
                           param_of=(po[rows] - p0).astype(np.int32), weight=None if wt is None else wt[rows],
                           grad=req.grad, dtype=req.dtype, part=("eval", p0, p1, rows))

        def rows_of(p0, p1):
            return np.sort(order[starts[p0]:starts[p1]])
        if len(order):
            one = int(order[0])
            limit = max(limit, self.cost(part(int(po[one]), int(po[one]) + 1, np.array([one]))) * (1.0 + 1e-9))
        p0 = 0
        while p0 < P:
            k = self._largest(lambda m: ok(part(p0, p0 + m, rows_of(p0, p0 + m)), limit), P - p0)
            if k:
                parts.append(part(p0, p0 + k, rows_of(p0, p0 + k)))
                p0 += k
                continue
            rows = rows_of(p0, p0 + 1)              # one parameter set over the limit: slices of its rows
            m = self._largest(lambda q: ok(part(p0, p0 + 1, rows[:q]), limit), len(rows))
            if not m:
                return None
            parts += [part(p0, p0 + 1, rows[i:i + m]) for i in range(0, len(rows), m)]
            p0 += 1
        return parts

    def finalize(self, req: Request, out):
        """The request's result from one launch's output."""
        if req.kind == "sample" and req.grad:
            out = dict(out)
            A, G = out.pop("A"), out.pop("G")
            out["grad"] = loo_score_gradient(A, G, out["cost"].sum(axis=1), int(req.samples))
        return out

    def combine(self, req: Request, outs):
        """The result of a split request from its parts' outputs, in part order."""
        P, K = req.n_params, np.asarray(req.theta).reshape(req.n_params, -1).shape[1]
        if req.kind == "sample":
            S = int(req.samples)
            first = next(o for o in outs if "samples" in o)
            samples = np.zeros((P, S) + first["samples"].shape[2:], dtype=first["samples"].dtype)
            cost = np.zeros((P, S)) if "cost" in first else None
            A = np.zeros((P, K)) if req.grad else None
            G = np.zeros((P, K)) if req.grad else None
            for u, o in zip(req.part["descs"], outs):
                _, p0, p1, c0, c1, s0, s1 = u
                if s1 < int(req.burn_in) + 1:
                    continue                       # an earlier slice of these chains' sweeps
                samples[p0:p1, c0:c1] = o["samples"].reshape((p1 - p0, c1 - c0) + samples.shape[2:])
                if cost is not None:
                    cost[p0:p1, c0:c1] = o["cost"].reshape(p1 - p0, c1 - c0)
                if req.grad:
                    A[p0:p1] += o["A"]
                    G[p0:p1] += o["G"]
            res = {"samples": samples}
            if cost is not None:
                res["cost"] = cost
            if req.grad:
                res["grad"] = loo_score_gradient(A, G, cost.sum(axis=1), S)
            return res
        B = req.n_rows
        res = {}
        for u, o in zip(req.part["descs"], outs):
            _, p0, p1, rows = u
            for k, v in o.items():
                if k == "grad":
                    res.setdefault("grad", np.zeros((P, K)))[p0:p1] += v
                else:
                    res.setdefault(k, np.zeros(B, dtype=v.dtype))[rows] = v
        return res

    # ---------------------------------------------------------- launch
    def _to_dev(self, a, dtype):
        t = self.torch.as_tensor(np.ascontiguousarray(a)).to(dtype).pin_memory()
        return t.to(self.device, non_blocking=True)

    def _to_host(self, t):
        h = self.torch.empty(t.shape, dtype=t.dtype, pin_memory=True)
        h.copy_(t, non_blocking=True)
        return h

    def launch(self, batch: List[Request], stream: int):
        torch, L = self.torch, self.L
        head = batch[0]
        g = self.graphs[head.graph]
        st = self.streams[stream]
        keep = []                                  # device tensors live until the event fires
        with torch.cuda.stream(st):
            if head.kind == "sample":
                out = self._launch_sample(g, head, keep)
            else:
                out = self._launch_eval(g, batch, keep)
            ev = torch.cuda.Event()
            ev.record(st)
        return (ev, out, keep)

    def _launch_sample(self, g, r: Request, keep):
        torch, L = self.torch, self.L
        P, S = r.n_params, int(r.samples)
        theta = self._to_dev(np.asarray(r.theta, dtype=np.float64).reshape(P, -1), torch.float64)
        chains = P * S
        ws = torch.empty(self.ws_bytes(g, r.dtype, chains, L.AC_OP_SAMPLE, r.share), dtype=torch.uint8,
                         device=self.device)
        edges = self.edges.get(r.graph)
        init, first = None, 0
        key = (r.graph, r.session)
        carry = None
        if r.parent is not None and r.part[1][0] == "sample":
            _, p0, _, c0, _, s0, s1 = r.part[1]
            carry = (r.parent.rid, p0, c0, s1 < int(r.parent.burn_in) + 1)
            if s0 > 0:
                with self._sess_lock:
                    init = self._carry.pop((r.parent.rid, p0, c0))
                first = s0
        if r.session is not None:
            with self._sess_lock:
                prev = self.sessions.get(key)
            if prev is not None and prev[2] == P and prev[3] == S:
                init, first = prev[0], prev[1]
                prev[4] = next(self._uses)
        more = carry is not None and carry[3]       # later slices resume these chains
        res = g.sample(theta, chains_per_param=S, samples_per_chain=1, burn_in=r.burn_in, thin=1,
                       seed=r.seed, cost_edges=edges, dtype=r.dtype, want_cost=edges is not None and not more,
                       want_states=r.grad or r.session is not None or more, validate=False, ws=ws,
                       init_states=init, first_sweep=first, chain_offset=r.chain_offset)
        keep += [theta, ws, res]
        if init is not None:
            keep.append(init)      # read on this stream: live until the launch completes
        if more:
            # the next slice is launched only after this one completes (the
            # scheduler orders them), so the states are final by then
            with self._sess_lock:
                self._carry[carry[:3]] = res["states"].reshape(chains, -1)
            return ("sample", {})
        if r.session is not None:
            # the chains' last states stay on the device for the next request
            with self._sess_lock:
                self.sessions[key] = [res["states"].reshape(chains, -1), first + r.burn_in + 1, P, S,
                                      next(self._uses)]
        out = {"samples": self._to_host(res["samples"])}
        if res["cost"] is not None:
            out["cost"] = self._to_host(res["cost"])
        if r.grad:
            if res["cost"] is None:
                raise ValueError(f"graph {r.graph!r} has no cost edges for a sampled gradient")
            # the sums the score-function estimate needs per parameter set:
            # A = sum_i C_i g_i and G = sum_i g_i with g_i = d log|f(s_i)|^2 / d theta
            # (combined with the leave-one-out baseline once all of a set's samples are in)
            states = res["states"].reshape(chains, -1)
            param_of = torch.arange(P, dtype=torch.int32, device=self.device).repeat_interleave(S)
            gws = torch.empty(self.ws_bytes(g, r.dtype, chains, L.AC_OP_GRAD, r.share), dtype=torch.uint8,
                              device=self.device)
            ones = torch.ones(chains, dtype=torch.float64, device=self.device)
            ga = g.grad(theta, states, param_of, mode="logprob", weight=res["cost"].reshape(-1), dtype=r.dtype,
                        validate=False, ws=gws)
            gg = g.grad(theta, states, param_of, mode="logprob", weight=ones, dtype=r.dtype, validate=False,
                        ws=gws)
            keep += [states, param_of, gws, ones, ga, gg]
            out["A"] = self._to_host(ga["grad"])
            out["G"] = self._to_host(gg["grad"])
        return ("sample", out)

    def _launch_eval(self, g, batch: List[Request], keep):
        torch, L = self.torch, self.L
        head = batch[0]
        info = g.info
        theta, ev, po, wt, spans = stack_eval_batch(batch, info["n_angles"], info["n_words"], head.grad)
        d_theta = self._to_dev(theta, torch.float64)
        d_ev = self._to_dev(ev.view(np.int64), torch.int64)
        d_po = self._to_dev(po, torch.int32)
        keep += [d_theta, d_ev, d_po]
        if head.grad:
            d_w = self._to_dev(wt, torch.float64)
            ws = torch.empty(self.ws_bytes(g, head.dtype, len(po), L.AC_OP_GRAD, head.share), dtype=torch.uint8,
                             device=self.device)
            res = g.grad(d_theta, d_ev, d_po, mode="prob", weight=d_w, dtype=head.dtype, want_amp=True,
                         validate=False, ws=ws)
            keep += [d_w, ws, res]
            host = {"amp": self._to_host(res["amp"]), "grad": self._to_host(res["grad"])}
        else:
            ws = torch.empty(self.ws_bytes(g, head.dtype, len(po), L.AC_OP_EVAL, head.share), dtype=torch.uint8,
                             device=self.device)
            amp, prob = g.eval(d_theta, d_ev, d_po, dtype=head.dtype, validate=False, ws=ws)
            keep += [ws, amp, prob]
            host = {"amp": self._to_host(amp), "prob": self._to_host(prob)}
        return ("eval", host, spans)

    def discard(self, req: Request):
        """Drop what a failed split request left on the device."""
        with self._sess_lock:
            for k in [k for k in self._carry if k[0] == req.rid]:
                del self._carry[k]

    # ---------------------------------------------------------- completion
    def done(self, handle) -> bool:
        return handle[0].query()

    def results(self, handle):
        _, out, _ = handle
        if out[0] == "sample":
            return [{k: v.numpy().copy() for k, v in out[1].items()}]
        _, host, spans = out
        res = []
        for p0, P, b0, B in spans:
            r = {k: v.numpy()[b0:b0 + B].copy() for k, v in host.items() if k != "grad"}
            if "grad" in host:
                r["grad"] = host["grad"].numpy()[p0:p0 + P].copy()
            res.append(r)
        return res
