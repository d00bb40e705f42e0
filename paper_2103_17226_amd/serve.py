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
     free; the head of the queue is never overtaken, so a large request
     cannot starve;
  3. merges an admitted amplitude request with later queued ones of the same
     graph, dtype and kind into one launch.  Parameter sets are stacked and
     every element keeps its own parameter row, so each request gets what it
     would get alone: the upward pass is elementwise, and gradient segments
     start on a 256-element boundary so that the fixed-order reduction adds
     the same terms in the same order (padding rows carry weight 0 and a
     parameter row of their own that is dropped).  Sampling requests run
     alone: their chains are numbered from 0 within the request, which is
     what makes them reproducible from the seed.  A sampling request of a
     session resumes the chains that session left on the device; requests of
     one session run one at a time, in arrival order, and the chain states
     count against the memory budget until the session is closed.

Requests that arrive while others are on the device therefore start as soon
as a stream and memory free up, and their kernels overlap on the device.
Submissions beyond ``max_queue`` waiting requests, larger than the whole
budget, or (with ``max_seconds``) estimated to occupy the device longer than
that, are rejected at once.

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
    # filled in by the server
    rid: int = -1
    t_arrive: float = 0.0
    t_start: float = 0.0
    t_launched: float = 0.0
    t_done: float = 0.0
    footprint: int = 0
    future: Future = field(default_factory=Future, repr=False)

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
    seconds`` if ``max_seconds`` is used.  ``launch``, ``done`` and
    ``results`` may raise; the requests of that batch then fail with the
    exception.  With ``request_timeout`` a launch still running that long
    after it started fails its requests with TimeoutError at once; its memory
    and stream return when the device finishes."""

    def __init__(self, executor, mem_budget: int, clock: Callable[[], float] = time.perf_counter,
                 max_queue: int = 1 << 30, max_merge: int = 64, max_seconds: Optional[float] = None,
                 request_timeout: Optional[float] = None, tick: float = 1e-4):
        if mem_budget <= 0:
            raise ValueError("mem_budget must be positive")
        self.ex = executor
        self.budget = int(mem_budget)
        self.clock = clock
        self.max_queue = int(max_queue)
        self.max_merge = max(1, int(max_merge))
        self.max_seconds = max_seconds
        self.request_timeout = request_timeout
        self.tick = tick
        self.queue: collections.deque = collections.deque()
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
        for callers that replay a schedule of arrivals."""
        req.rid = next(self._ids)
        req.t_arrive = self.clock() if t_arrive is None else float(t_arrive)
        req.footprint = int(self.ex.footprint(req))
        if req.footprint > self.budget:
            self.rejected_memory += 1
            req.future.set_exception(AdmissionError(
                f"request needs {req.footprint} bytes of device memory, the budget is {self.budget}"))
            return req.future
        if self.max_seconds is not None:
            est = float(self.ex.cost(req))
            if est > self.max_seconds:
                self.rejected_cost += 1
                req.future.set_exception(AdmissionError(
                    f"request would hold the device ~{est:.3g} s, the limit is {self.max_seconds:.3g} s"))
                return req.future
        with self.lock:
            if len(self.queue) >= self.max_queue:
                self.rejected_queue += 1
                req.future.set_exception(AdmissionError(f"queue full ({self.max_queue} waiting)"))
                return req.future
            self.queue.append(req)
        return req.future

    def cancel(self, fut: Future) -> bool:
        """Cancel a request that is still waiting; one already on the device
        runs to completion (returns False)."""
        with self.lock:
            for r in self.queue:
                if r.future is fut:
                    self.queue.remove(r)
                    self.cancelled += 1
                    fut.cancel()
                    return True
        return False

    def start(self):
        if self.thread is not None:
            raise RuntimeError("server already started")
        self._stop.clear()
        self.thread = threading.Thread(target=self._run, name="ac-serve", daemon=True)
        self.thread.start()

    def idle(self) -> bool:
        with self.lock:
            return not self.queue and not self.inflight and not self.launching

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
            while self.queue:
                r = self.queue.popleft()
                self.cancelled += 1
                r.future.cancel()

    # ------------------------------------------------------------ scheduler
    def _fail(self, reqs, exc):
        for r in reqs:
            r.t_done = self.clock()
            self.failed += 1
            if not r.future.done():
                r.future.set_exception(exc)

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
                    r.t_done = now
                    self.completed.append(r)
                    r.future.set_result(o)
                    finished += 1
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

    def _session_busy(self, r: Request) -> bool:
        return r.session is not None and (r.graph, r.session) in self.busy_sessions

    def _take_batch(self):
        """Pop the next launch if it fits; called with the lock held.  The
        first request whose session is idle leads (requests of a busy session
        keep their place); later requests never overtake it for memory."""
        if not self.queue or not self.free_streams:
            return None
        idx = next((k for k, r in enumerate(self.queue) if not self._session_busy(r)), None)
        if idx is None:
            return None
        head = self.queue[idx]
        resident = self.ex.resident_bytes() if hasattr(self.ex, "resident_bytes") else 0
        if self.used + resident + head.footprint > self.budget:
            return None
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
    def latency_stats(self, since: float = float("-inf")) -> Dict[str, Any]:
        """Latency (arrival to completion) over requests that arrived at or
        after ``since``, with counts of every outcome."""
        done = [r for r in self.completed if r.t_arrive >= since]
        lat = np.array([r.t_done - r.t_arrive for r in done])
        out: Dict[str, Any] = {"completed": len(done), "failed": self.failed,
                               "rejected_memory": self.rejected_memory,
                               "rejected_queue": self.rejected_queue, "rejected_cost": self.rejected_cost, "timed_out": self.timed_out,
                               "cancelled": self.cancelled,
                               "launches": self.launches, "merged": self.merged,
                               "max_inflight": self.max_inflight, "peak_bytes": self.peak_used}
        if len(lat):
            out.update(p50_ms=float(np.percentile(lat, 50) * 1e3),
                       p99_ms=float(np.percentile(lat, 99) * 1e3),
                       mean_ms=float(lat.mean() * 1e3))
        return out


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
    shared, and launches of one graph overlap)."""

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
        self.sessions = {}        # (graph, session) -> [states [P*S, W] int64 on device, next sweep, P, S]
        self._sess_lock = threading.Lock()
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
            ws = g.workspace_size(req.dtype, chains, L.AC_OP_SAMPLE)
            nwq = (info["n_qubits"] + 63) // 64
            io = chains * 8 * (nwq + 1) + P * K * 8
            if req.grad:
                ws = max(ws, g.workspace_size(req.dtype, chains, L.AC_OP_GRAD))
                io += chains * (8 * W + 4 + 8 + cs) + P * K * 8
            return ws + io
        B = padded_rows(req.n_rows, req.grad)
        op = L.AC_OP_GRAD if req.grad else L.AC_OP_EVAL
        ws = g.workspace_size(req.dtype, B, op)
        return ws + B * (8 * W + 4 + 8 + cs) + (P + 1) * K * 16

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
        three with a gradient."""
        g = self.graphs[req.graph]
        info = g.info
        N = float(info["n_internal"])
        if req.kind == "sample":
            chains = req.n_params * int(req.samples)
            steps = 3.0 * N * (req.burn_in + 1) * (info["n_qubits"] // 2 + 1)
            if req.grad:
                steps += 3.0 * N
            kind, conc = g.sample_shape(req.dtype, chains)
            groups = -(-chains // max(conc, 1))
            lat = groups * steps * self.NODE_STEP_LATENCY[kind]
            return max(lat, chains * steps / self.NODE_STEP_RATE["sample"])
        passes = 3.0 if req.grad else 1.0
        lat = passes * N * self.NODE_STEP_LATENCY["eval"]
        return max(lat, req.n_rows * passes * N / self.NODE_STEP_RATE["eval"])

    def resident_bytes(self) -> int:
        """Device bytes of the resident session chains."""
        with self._sess_lock:
            return sum(int(v[0].numel()) * 8 for v in self.sessions.values())

    def drop_session(self, graph: str, session: str):
        with self._sess_lock:
            self.sessions.pop((graph, session), None)

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
        ws = torch.empty(max(g.workspace_size(r.dtype, chains, L.AC_OP_SAMPLE), 256), dtype=torch.uint8,
                         device=self.device)
        edges = self.edges.get(r.graph)
        init, first = None, 0
        key = (r.graph, r.session)
        if r.session is not None:
            with self._sess_lock:
                prev = self.sessions.get(key)
            if prev is not None and prev[2] == P and prev[3] == S:
                init, first = prev[0], prev[1]
        res = g.sample(theta, chains_per_param=S, samples_per_chain=1, burn_in=r.burn_in, thin=1,
                       seed=r.seed, cost_edges=edges, dtype=r.dtype, want_cost=edges is not None,
                       want_states=r.grad or r.session is not None, validate=False, ws=ws,
                       init_states=init, first_sweep=first)
        keep += [theta, ws, res]
        if init is not None:
            keep.append(init)      # read on this stream: live until the launch completes
        if r.session is not None:
            # the chains' last states stay on the device for the next request
            with self._sess_lock:
                self.sessions[key] = [res["states"].reshape(chains, -1), first + r.burn_in + 1, P, S]
        out = {"samples": self._to_host(res["samples"])}
        if res["cost"] is not None:
            out["cost"] = self._to_host(res["cost"])
        if r.grad:
            if res["cost"] is None:
                raise ValueError(f"graph {r.graph!r} has no cost edges for a sampled gradient")
            # score-function estimate: d<C>/dtheta = E[(C - mean C) d log P / dtheta]
            cost = res["cost"]
            wgt = ((cost - cost.mean(dim=1, keepdim=True)) / S).reshape(-1).contiguous()
            states = res["states"].reshape(chains, -1)
            param_of = torch.arange(P, dtype=torch.int32, device=self.device).repeat_interleave(S)
            gws = torch.empty(max(g.workspace_size(r.dtype, chains, L.AC_OP_GRAD), 256), dtype=torch.uint8,
                              device=self.device)
            gr = g.grad(theta, states, param_of, mode="logprob", weight=wgt, dtype=r.dtype, validate=False,
                        ws=gws)
            keep += [wgt, states, param_of, gws, gr]
            out["grad"] = self._to_host(gr["grad"])
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
            ws = torch.empty(max(g.workspace_size(head.dtype, len(po), L.AC_OP_GRAD), 256), dtype=torch.uint8,
                             device=self.device)
            res = g.grad(d_theta, d_ev, d_po, mode="prob", weight=d_w, dtype=head.dtype, want_amp=True,
                         validate=False, ws=ws)
            keep += [d_w, ws, res]
            host = {"amp": self._to_host(res["amp"]), "grad": self._to_host(res["grad"])}
        else:
            ws = torch.empty(max(g.workspace_size(head.dtype, len(po), L.AC_OP_EVAL), 256), dtype=torch.uint8,
                             device=self.device)
            amp, prob = g.eval(d_theta, d_ev, d_po, dtype=head.dtype, validate=False, ws=ws)
            keep += [ws, amp, prob]
            host = {"amp": self._to_host(amp), "prob": self._to_host(prob)}
        return ("eval", host, spans)

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
