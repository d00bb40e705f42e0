"""Benchmark of the batched arithmetic-circuit hot path on one MI355X.

Workload (default): noisy QAOA p=1 MaxCut on a seeded random 3-regular graph
with 8 qubits and a depolarizing channel (p = 0.01) after every gate; 1024
parameter sets (gamma, beta) ~ U[0, 2pi)^2, 1000 Gibbs samples each
(1000 independent chains per parameter set, one sample per chain after the
burn-in), complex64 DAG arithmetic with FP64 weights, probabilities and
reductions.

One step = one pass of the whole hot path over that batch:
  1. ac_sample: weight-slot table, evidence decode, upward pass, downward
     pass and Gibbs decisions, repeated on device until every chain has its
     sample; emits the sampled states and their MaxCut cost;
  2. ac_grad_batch over the 1,024,000 sampled states in LOGPROB mode with the
     cost as weight: upward + downward pass, chain rule and the per-parameter
     FP64 reduction, i.e. the score-function estimate of d<C>/d theta
     (times the sample count).

Serving leg (after the timed steps, reported under "serving"): the
serving mix -- a pool of noisy QAOA circuits (p in {1,2}, n in
{6,8,12,16,20}, 4 seeded 3-regular graphs each, depolarizing strength ~
U[1e-3,1e-2] per circuit), Poisson arrivals, per request a circuit uniform
from the pool, P ~ log-uniform{1..256} parameter sets, an amplitude request
(64 outputs per set) w.p. 0.1 else S ~ log-uniform{1..4096} samples per set,
a gradient w.p. 0.5 -- through the continuous-batching loop at 200, 500,
1000 and 2000 req/s (10 s warm-up and 60 s measured at 2000 req/s, 5 s and
15 s at the lower rates);
requests estimated to hold the device over 0.5 s are split into parts; 12
streams, each on a hardware queue of its own (the process asks for 16); p50/p99
latency from arrival to completion, throughput (requests completed inside the
measured window per second) and outcomes per offered rate, and the admission
estimate against requests run alone.
The pool (all 40 circuits; the p=2, n=20 ones compile to ACs of about a
million nodes) compiles in worker processes while the other legs run, with
a blob cache on disk; --serve-pool fast leaves the n=20, p=2 circuits out.

Prints one JSON line.  --gpus > 1 is refused: the library runs on one GPU.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "AC node-evals/s & samples/s vs plain at 1e-5 rel tol; serving p50/p99 latency"
HBM_PEAK_GBS = 8000.0
KERNELS = os.path.join(ROOT, "paper_2103_17226_amd", "csrc", "qkc_kernels.hip")

# HBM bytes per dispatch from rocprofv3 FETCH_SIZE / WRITE_SIZE runs (scaled by
# the copy-kernel calibration, FETCH x 2.0, WRITE x 1.0), valid only for the
# kernel source and the AC they were taken on, and the default workload of
# each leg.
PROFILED_TRAFFIC = {
    "k_sample_stream": {"kernel_sha256_16": "22605b8be4dbf50d", "ac_sha256_16": "d3190d478a0e63f4",
                        "bytes": 1777647754240,
                        "profile": "profiles/k_sample_stream_qaoa_n8_p1_dep.md"},
    "k_eval": {"kernel_sha256_16": "22605b8be4dbf50d", "ac_sha256_16": "53555d81365c02e0",
               "bytes": 93752513536,
               "profile": "profiles/k_eval_qaoa_n16_p2_dep_ad.md"},
}


def _sha16(data: bytes) -> str:
    import hashlib
    return hashlib.sha256(data).hexdigest()[:16]


def kernel_sha16() -> str:
    with open(KERNELS, "rb") as f:
        return _sha16(f.read())


def profiled_traffic(kernel: str, default_workload: bool, blob: bytes):
    """Profiled bytes per dispatch, or None if the kernel source, the AC or
    the workload differ from the profiled ones."""
    ent = PROFILED_TRAFFIC.get(kernel)
    if ent is None or not default_workload:
        return None
    if kernel_sha16() != ent["kernel_sha256_16"] or _sha16(blob) != ent["ac_sha256_16"]:
        return None
    return ent["bytes"]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--burn-in", type=int, default=10)
    ap.add_argument("--params", type=int, default=1024)
    ap.add_argument("--chains", type=int, default=1000)
    ap.add_argument("--dtype", default="c64")
    ap.add_argument("--order-trials", type=int, default=64,
                    help="greedy elimination-order runs the compiler picks from")
    ap.add_argument("--compiler", choices=["ve", "dpll"], default="dpll",
                    help="AC compiler of the sampling and gradient workloads: variable elimination "
                         "or the search-based (decision-DNNF) compiler")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-eval", action="store_true")
    ap.add_argument("--eval-steps", type=int, default=5)
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--mpe-params", type=int, default=4096, help="angle pairs of the MPE leg (16 outcomes each)")
    ap.add_argument("--serve-rates", default="200,500,1000,2000",
                    help="offered request rates (req/s), one serving run each")
    ap.add_argument("--serve-seconds", type=float, default=60.0,
                    help="measured window at the highest offered rate")
    ap.add_argument("--serve-seconds-low", type=float, default=15.0,
                    help="measured window at the lower offered rates")
    ap.add_argument("--serve-warmup", type=float, default=10.0,
                    help="warm-up before the measured window at the highest offered rate")
    ap.add_argument("--serve-warmup-low", type=float, default=5.0)
    ap.add_argument("--serve-drain", type=float, default=15.0,
                    help="seconds to let requests in flight finish after the last arrival")
    ap.add_argument("--serve-pool", choices=["fast", "full"], default="full")
    ap.add_argument("--blob-cache", default=os.path.join(os.path.expanduser("~"), ".cache", "qkc_blobs"),
                    help="directory of cached compiled serving-pool blobs ('' for none)")
    ap.add_argument("--serve-streams", type=int, default=12)
    ap.add_argument("--serve-hw-queues", type=int, default=16,
                    help="hardware queues of this process (GPU_MAX_HW_QUEUES, read when HIP starts; at most 32): "
                         "at least one per serving stream, so a short launch never waits behind a long kernel "
                         "on a shared queue")
    ap.add_argument("--serve-queue", type=int, default=16)
    ap.add_argument("--serve-part-streams", type=int, default=1,
                    help="streams the parts of split requests hold at once, in total")
    ap.add_argument("--serve-part-share", type=float, default=0.5,
                    help="share of the device's workgroups a part of a split request runs on")
    ap.add_argument("--serve-max-split", type=int, default=4, help="split requests waiting or running at once")
    ap.add_argument("--serve-split-backlog", type=float, default=30.0,
                    help="estimated device seconds of waiting parts beyond which split requests are refused")
    ap.add_argument("--serve-budget-gib", type=float, default=64.0)
    ap.add_argument("--serve-max-seconds", type=float, default=0.5,
                    help="split requests estimated to hold the device longer than this into parts")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only copy 1 GiB device-to-device three times (calibrates the HBM "
                         "byte counters of a profiler run) and exit")
    return ap.parse_args()


def copy_peak_gbs(dev) -> float:
    """Achievable HBM bandwidth on this device: a 1 GiB elementwise copy
    kernel (b = a * 1; read + write = 2 GiB of traffic per copy), best of
    three timed batches of five copies, HIP events on the current stream.
    (torch's copy_ reaches less: 5.1 TB/s against 6.2 TB/s measured.)"""
    import torch
    a = torch.empty(1 << 28, dtype=torch.float32, device=dev)
    b = torch.empty_like(a)
    a.fill_(1.0)
    torch.mul(a, 1.0, out=b)
    torch.cuda.synchronize()
    best = 0.0
    for _ in range(3):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(5):
            torch.mul(a, 1.0, out=b)
        e1.record()
        torch.cuda.synchronize()
        best = max(best, 5 * 2 * (1 << 30) / (e0.elapsed_time(e1) / 1e3) / 1e9)
    del a, b
    torch.cuda.empty_cache()
    return best


def copy_probe():
    import torch
    a = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes": 3 * (1 << 30)}))


def compile_pool_start(full: bool, cache_dir: str):
    """Start compiling the serving pool in worker processes (spawned before
    this process touches the GPU), largest circuits first, so that it runs
    while the GPU legs do; returns (pool, executor, futures, start time).
    Blobs are cached on disk under cache_dir (keyed by the circuit and the
    compiler's source), so a second run on the same machine loads them."""
    import multiprocessing as mp
    from concurrent.futures import ProcessPoolExecutor

    import workloads as W
    from paper_2103_17226_amd.blob import compile_blob_cached
    pool = W.serving_pool()
    if not full:
        pool = [c for c in pool if not (c.n >= 20 and c.n_angles == 4)]
    t0 = time.perf_counter()
    workers = max(1, min(16, (os.cpu_count() or 1)))
    ex = ProcessPoolExecutor(workers, mp_context=mp.get_context("spawn"))
    order = sorted(range(len(pool)), key=lambda i: -(pool[i].n * pool[i].n_angles))
    # both compilers for the circuits up to 16 qubits (the smaller AC serves;
    # the search compiler takes minutes on the 20-qubit p=2 ones)
    futs = {i: ex.submit(compile_blob_cached, pool[i], cache_dir, method="best" if pool[i].n <= 16 else "ve")
            for i in order}
    return pool, ex, [futs[i] for i in range(len(pool))], t0


def compile_pool_finish(started):
    pool, ex, futs, t0 = started
    out = [f.result() for f in futs]
    ex.shutdown()
    blobs = [b for b, _ in out]
    return pool, blobs, time.perf_counter() - t0, sum(1 for _, hit in out if hit)


def estimate_check(graphs, pool, args, n=40, budget_s=20.0):
    """The admission estimate against each request's service time when it
    runs alone (one stream, nothing else on the device): requests of the
    serving mix that the server would launch whole, each launched twice and
    the second launch timed from launch to completion (inputs staged from
    the host, results copied back).  Under load the same ratio also holds
    the time a launch waits for compute units behind the other streams."""
    import numpy as np
    import torch

    import workloads as W
    from paper_2103_17226_amd.serve import GraphExecutor, Request
    edges = {c.name: c.edges for c in pool}
    ex = GraphExecutor(graphs, edges, n_streams=1)
    reqs = W.serving_requests(pool, 50.0, 10.0, seed=W.sub_seed("arrivals", 5) + 7919)
    rows, t_all = [], time.perf_counter()
    for r in reqs:
        if len(rows) >= n or time.perf_counter() - t_all > budget_s:
            break
        q = Request(graph=pool[r["circuit"]].name, theta=r["theta"], evidence=r.get("evidence"),
                    param_of=r.get("param_of"), weight=r.get("weight"), samples=r["samples"], grad=r["grad"],
                    burn_in=10, seed=r["seed"])
        q.rid = len(rows)
        est = ex.cost(q)
        if est > args.serve_max_seconds:
            continue
        for rep in range(2):
            torch.cuda.synchronize()
            t = time.perf_counter()
            h = ex.launch([q], 0)
            h[0].synchronize()
            ex.results(h)
            dt = time.perf_counter() - t
        rows.append((dt / est, dt, est, q.kind, graphs[q.graph].info["n_internal"]))
    del ex
    torch.cuda.synchronize()
    if not rows:
        return None
    ratio = np.array([x[0] for x in rows])
    return {"requests": len(rows), "ratio_p50": float(np.median(ratio)), "ratio_min": float(ratio.min()),
            "ratio_max": float(ratio.max()),
            "ratio_p50_above_10ms": (float(np.median([x[0] for x in rows if x[1] > 0.01]))
                                     if any(x[1] > 0.01 for x in rows) else None),
            "service_ms_p50": float(np.median([x[1] for x in rows]) * 1e3),
            "est_ms_p50": float(np.median([x[2] for x in rows]) * 1e3)}


def serve_run(graphs, pool, rate, args):
    """One serving run at an offered rate; returns its summary (requests
    that arrive in the warm-up window are served but not counted)."""
    import numpy as np
    import torch

    import workloads as W
    from paper_2103_17226_amd.serve import GraphExecutor, Request, Server
    edges = {c.name: c.edges for c in pool}
    ex = GraphExecutor(graphs, edges, n_streams=args.serve_streams)
    srv = Server(ex, mem_budget=int(args.serve_budget_gib * (1 << 30)), max_queue=args.serve_queue,
                 max_seconds=args.serve_max_seconds, part_streams=args.serve_part_streams,
                 part_share=args.serve_part_share, max_split=args.serve_max_split,
                 split_backlog=args.serve_split_backlog)
    top = rate >= max(float(x) for x in args.serve_rates.split(",") if x)
    seconds = args.serve_seconds if top else args.serve_seconds_low
    warmup = args.serve_warmup if top else args.serve_warmup_low
    total = warmup + seconds
    reqs = W.serving_requests(pool, rate, total, seed=W.sub_seed("arrivals", 5) + int(rate))
    srv.start()
    t0 = time.perf_counter()
    futs = []
    next_note = 10.0
    for r in reqs:
        delay = t0 + r["t"] - time.perf_counter()
        if delay > 0:
            time.sleep(delay)
        if r["t"] >= next_note:
            print(f"#   t={r['t']:.0f} s ({time.perf_counter() - t0:.0f} s elapsed): {len(futs)} submitted, "
                  f"{len(srv.completed)} completed", file=sys.stderr, flush=True)
            next_note += 10.0
        q = Request(graph=pool[r["circuit"]].name, theta=r["theta"], evidence=r.get("evidence"),
                    param_of=r.get("param_of"), weight=r.get("weight"), samples=r["samples"], grad=r["grad"],
                    burn_in=10, seed=r["seed"])
        srv.submit(q, t_arrive=t0 + r["t"])
        futs.append(q)
    t_end = time.perf_counter()
    srv.stop(drain=True, timeout=args.serve_drain)
    print(f"#   drained: {len(srv.completed)} completed", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    since = t0 + warmup
    st = srv.latency_stats(since=since)
    window = [q for q in futs if q.t_arrive >= since]

    def outcome(q):
        f = q.future
        if f.cancelled() or not f.done():
            return "unfinished"
        e = f.exception()
        if e is None:
            return "completed"
        msg = str(e)
        if "queue full" in msg:           # whole requests, or the split requests' backlog
            return "rejected_queue"
        if "hold the device" in msg:
            return "rejected_cost"
        if "device memory" in msg or "resident" in msg:
            return "rejected_memory"
        if "at least 2 samples" in msg:
            return "rejected_invalid"
        return "failed"

    counts = {k: 0 for k in ("completed", "rejected_queue", "rejected_cost", "rejected_memory", "rejected_invalid",
                             "failed", "unfinished")}
    for q in window:
        counts[outcome(q)] += 1
    ok = [q for q in window if outcome(q) == "completed"]
    # steady-state rate: requests of any arrival time completed inside the
    # measured window (a split request finishing in the drain does not
    # stretch the window)
    span = t_end - since
    done_in = [q for q in futs if outcome(q) == "completed" and since <= q.t_done <= t_end]
    # how the admission estimate compares with the time each request held a stream
    ratio = [(q.t_done - q.t_start) / max(ex.cost(q), 1e-6) for q in ok if not isinstance(q.part, dict)]
    stuck = [{"graph": q.graph, "kind": q.kind, "P": q.n_params, "S": q.samples, "rows": q.n_rows,
              "grad": q.grad, "est_s": ex.cost(q)} for q in window if outcome(q) == "unfinished"]
    out = {"offered_rps": rate, "warmup_s": warmup, "measured_s": seconds, "arrivals": len(window),
           **counts, "split_requests": st["split_requests"], "split_parts": st["split_parts"],
           "p50_ms": st.get("p50_ms"), "p99_ms": st.get("p99_ms"), "mean_ms": st.get("mean_ms"),
           "whole_requests": st["whole"], "split_requests_latency": st["split"],
           "completed_in_window": len(done_in),
           "throughput_rps": len(done_in) / span,
           "samples_per_s": sum(q.n_params * q.samples for q in done_in) / span,
           "amplitudes_per_s": sum(q.n_rows for q in done_in) / span,
           "launches": st["launches"], "merged": st["merged"], "max_inflight": st["max_inflight"],
           "peak_gib": st["peak_bytes"] / (1 << 30),
           "launch_host_ms_p50": float(np.median([(q.t_launched - q.t_start) * 1e3 for q in ok])) if ok else None,
           "queue_wait_ms_p50": float(np.median([(q.t_start - q.t_arrive) * 1e3 for q in ok])) if ok else None,
           "service_over_estimate_p50": float(np.median(ratio)) if ratio else None,
           "service_over_estimate_max": float(max(ratio)) if ratio else None,
           "unfinished_requests": stuck[:5]}
    if len(ok) <= 16:       # light load: every request's estimate and timeline
        out["requests"] = [{"graph": q.graph, "ac_nodes": graphs[q.graph].info["n_internal"], "kind": q.kind,
                            "P": q.n_params, "S": q.samples, "rows": q.n_rows, "grad": q.grad,
                            "est_ms": ex.cost(q) * 1e3, "queue_ms": (q.t_start - q.t_arrive) * 1e3,
                            "host_ms": (q.t_launched - q.t_start) * 1e3, "device_ms": (q.t_done - q.t_launched) * 1e3}
                           for q in ok]
    return out


def byte_model(comp, W: int, cs: int):
    """Bytes of the streaming model on the compiled DAG for one element:
    upward pass (every node value written once, every internal child read
    once, the evidence words read once, the amplitude written) and downward
    pass (node values and parent adjoints read, every adjoint written)."""
    tags = comp.col >> 30
    E_ii = int((tags == 0).sum())
    N = comp.n_internal
    up = cs * (E_ii + N) + 8 * W + cs
    down = cs * (N + 2 * E_ii)
    return up, down, E_ii


def plan_byte_model(info, cs: int):
    """The same streaming model on the sum-of-products plan the kernels run
    (products folded into their sum parents never get a row): per element,
    upward pass s*(super-nodes + super-node factors) + evidence words + the
    amplitude; downward pass s*(super-nodes + adjoint and sibling rows read);
    leaf step s*(adjoint and sibling rows read + one derivative per value)."""
    S = info["n_super"]
    up = cs * (S + info["n_super_node_factors"]) + 8 * info["n_words"] + cs
    down = cs * (S + info["n_super_down_reads"])
    leaf = cs * (info["n_super_leaf_reads"] + info["n_indicator_leaves"])
    return up, down, leaf


_AC_CACHE = {}


def compile_ac(circ, method: str, order_trials: int = 64):
    """The AC of a workload circuit from the chosen compiler (compiled once
    per run: the GPU legs and the CPU baseline use the same AC)."""
    key = (circ.name, len(circ.ops), method, order_trials)
    if key not in _AC_CACHE:
        if method == "dpll":
            from paper_2103_17226_amd.dnnf import compile_circuit_dpll
            _AC_CACHE[key] = compile_circuit_dpll(circ)
        else:
            from paper_2103_17226_amd.compiler import compile_circuit
            _AC_CACHE[key] = compile_circuit(circ, order_trials=order_trials)
    return _AC_CACHE[key]


def eval_leg(args, circ_cfg):
    """Amplitudes and gradients over the batch of the 16-qubit p=2 workload:
    4096 parameter sets x 64 seeded (x, k) with k from the channel priors."""
    import numpy as np
    import torch

    from paper_2103_17226_amd import _lib
    from paper_2103_17226_amd.api import ACGraph
    t0 = time.perf_counter()
    comp = compile_ac(circ_cfg["circuit"], args.compiler)
    t_comp = time.perf_counter() - t0
    g = ACGraph(comp, device=0)
    dev = g.torch_device
    theta = torch.as_tensor(circ_cfg["theta"], device=dev)
    ev = torch.as_tensor(circ_cfg["evidence"].view(np.int64), device=dev)
    po = torch.as_tensor(circ_cfg["param_of"], device=dev)
    B = ev.shape[0]
    info = g.info
    ws_e = g.workspace("c64", B, _lib.AC_OP_EVAL)
    wgt = torch.ones(B, dtype=torch.float64, device=dev)

    def timed(fn, n):
        fn()
        torch.cuda.synchronize()
        evs = []
        for _ in range(n):
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record()
            fn()
            b.record()
            evs.append((a, b))
        torch.cuda.synchronize()
        return float(np.mean([a.elapsed_time(b) for a, b in evs])) / 1e3

    t_eval = timed(lambda: g.eval(theta, ev, po, dtype="c64", validate=False, ws=ws_e), args.eval_steps)
    t_grad = timed(lambda: g.grad(theta, ev, po, mode="prob", weight=wgt, dtype="c64", validate=False),
                   args.eval_steps)
    # the differentiated form against the plain batched evaluation (same amplitudes expected)
    a_eval, _ = g.eval(theta, ev, po, dtype="c64", validate=False, ws=ws_e)
    a_grad = g.grad(theta, ev, po, mode="prob", weight=wgt, dtype="c64", validate=False, want_amp=True)["amp"]
    diff = (a_grad - a_eval).abs() / a_eval.abs().clamp_min(1e-30)
    grad_vs_eval = float(diff.max().item())
    del a_eval, a_grad, diff
    dag_up, dag_down, E_ii = byte_model(comp, info["n_words"], 8)
    up, _, _ = plan_byte_model(info, 8)
    N = info["n_internal"]
    achieved = up * B / t_eval / 1e9
    # complex64 against complex128 per result, on the first 32768 elements
    sub = slice(0, 32768)
    _, p64 = g.eval(theta, ev[sub], po[sub], dtype="c64", validate=False)
    _, p128 = g.eval(theta, ev[sub], po[sub], dtype="c128", validate=False)
    p64, p128 = p64.cpu().numpy(), p128.cpu().numpy()
    rel = np.abs(p64 - p128) / np.maximum(p128, 1e-300)
    big = p128 >= 1e-3 * p128.max()
    out = {
        "workload": "noisy QAOA p=2 MaxCut, seeded random 3-regular graph, 16 qubits, depolarizing "
                    "p_c~U[1e-3,1e-2] + amplitude damping 5e-3 after every gate; 4096 angle sets x 64 "
                    "seeded (x,k) = 262,144 amplitudes, c64 with FP64 |f|^2",
        "ac_internal_nodes": N, "ac_edges": info["n_edges"], "ac_levels": info["n_levels"],
        "ac_compiler": args.compiler, "ac_super_nodes": info["n_super"], "compile_s": t_comp, "batch": B,
        "eval_ms": t_eval * 1e3, "amplitudes_per_s": B / t_eval, "node_evals_per_s": N * B / t_eval,
        "grad_ms": t_grad * 1e3, "grad_elements_per_s": B / t_grad,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "kernel": "k_eval (upward pass, sum-of-products plan)",
                     "bytes_per_element": up, "ac_super_nodes": info["n_super"],
                     "dag_model_bytes_per_element": dag_up,
                     "dag_model_GBps": dag_up * B / t_eval / 1e9,
                     "traffic": profiled_traffic("k_eval", circ_cfg["evidence"].shape[0] == 262144, g.blob),
                     "kernel_sha256_16": kernel_sha16(), "ac_sha256_16": _sha16(g.blob),
                     "traffic_unit": "HBM bytes per dispatch (rocprofv3)"},
        "grad_model_GBps": (dag_up + dag_down) * B / t_grad / 1e9,
        "grad_vs_eval_amplitude_max_rel_diff": grad_vs_eval,
        "c64_vs_c128_branch_prob_rel_err": {"max": float(rel[big].max()), "p99": float(np.percentile(rel[big], 99)),
                                            "median": float(np.median(rel[big])), "results": int(big.sum())},
    }
    g.close()
    del ws_e
    torch.cuda.empty_cache()
    return out


def mpe_leg(steps: int, P: int = 4096):
    """Most probable noise events (max-product pass, complex128) for every
    outcome of a 4-qubit ring QAOA with 8 channels, P angle pairs x 16
    outcomes per call."""
    import numpy as np
    import torch

    import workloads as W
    from paper_2103_17226_amd.api import ACGraph
    from paper_2103_17226_amd.dnnf import compile_circuit_dpll
    circ = W.qaoa_ring_mpe(4)
    t0 = time.perf_counter()
    ac = compile_circuit_dpll(circ, mpe=True)
    t_comp = time.perf_counter() - t0
    g = ACGraph(ac, device=0)
    dev = g.torch_device
    n = circ.n
    theta = torch.as_tensor(W.uniform_angles(P, circ.n_angles, W.sub_seed("angles", 7)), device=dev)
    vals = np.zeros((P << n, circ.n_vars), dtype=np.int64)
    vals[:, :n] = np.tile([[(x >> q) & 1 for q in range(n)] for x in range(1 << n)], (P, 1))
    ev = torch.as_tensor(W.pack_evidence(circ, vals).view(np.int64), device=dev)
    po = torch.arange(P, dtype=torch.int32, device=dev).repeat_interleave(1 << n)
    B = ev.shape[0]
    ws = g.workspace("c128", B, 3)
    g.mpe(theta, ev, po, validate=False, ws=ws)
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(steps):
        prob, _ = g.mpe(theta, ev, po, validate=False, ws=ws)
    b.record()
    torch.cuda.synchronize()
    t = a.elapsed_time(b) / steps / 1e3
    N, E = g.info["n_internal"], g.info["n_edges"]
    tags = ac.col >> 30
    e_ii = int((tags == 0).sum())
    up = 16 * (e_ii + N) + 8 * g.info["n_words"]          # upward pass, complex128 rows
    out = {"workload": "most probable noise events of every outcome: QAOA p=1, 4-ring, amplitude damping "
                       f"0.05 after each H, depolarizing 0.02 after each RX (8 channels); {P} angle pairs x "
                       "16 outcomes, complex128",
           "ac_internal_nodes": N, "ac_edges": E, "ac_levels": g.info["n_levels"], "compile_s": t_comp,
           "queries": B, "ms_per_call": t * 1e3, "queries_per_s": B / t, "node_evals_per_s": N * B / t,
           "upward_model_GBps": up * B / t / 1e9,
           "mean_best_probability": float(prob.mean().item())}
    g.close()
    return out


def small_configs_leg(steps: int):
    """The remaining workloads: the 4-qubit ring (64 angle pairs x all 16
    outputs, complex128, launch-bound), the noise-free 32-qubit circuit
    (256 angle pairs x 3907 Gibbs chains = 1,000,192 samples, complex64) and,
    beyond the configurations, its p=2 version (8,192 chains, 10 sweeps)."""
    import numpy as np
    import torch

    import workloads as W
    from paper_2103_17226_amd.api import ACGraph

    def timed(fn, n):
        fn()
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(n):
            fn()
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) / n / 1e3

    c1 = W.config(1)
    g1 = ACGraph(c1["circuit"], device=0)
    dev = g1.torch_device
    th1 = torch.as_tensor(c1["theta"], device=dev)
    ev1 = torch.as_tensor(c1["evidence"].view(np.int64), device=dev)
    po1 = torch.as_tensor(c1["param_of"], device=dev)
    t1 = timed(lambda: g1.eval(th1, ev1, po1, dtype="c128", validate=False), 50)
    c4 = W.config(4)
    g4 = ACGraph(c4["circuit"], device=0)
    th4 = torch.as_tensor(c4["theta"], device=dev)
    C = c4["chains_per_param"]
    t4 = timed(lambda: g4.sample(th4, C, 1, 10, 1, 7, dtype="c64", validate=False), steps)
    out = {
        "ring4_eval_us_per_call": t1 * 1e6, "ring4_amplitudes_per_s": ev1.shape[0] / t1,
        "ring4_batch": int(ev1.shape[0]),
        "qaoa_n32_samples_per_s": th4.shape[0] * C / t4, "qaoa_n32_sample_ms": t4 * 1e3,
        "qaoa_n32_chains": int(th4.shape[0] * C), "qaoa_n32_ac_nodes": g4.info["n_internal"],
    }
    g1.close()
    g4.close()
    # the paper's largest QAOA setting, noise-free p=2 on 32 qubits: a small
    # batch (2 angle sets x 4096 chains) on a large AC, one timed call
    from paper_2103_17226_amd.compiler import compile_circuit
    circ = W.qaoa_maxcut(32, W.random_regular_graph(32, 3, W.sub_seed("graph", 4)), 2)
    t0 = time.perf_counter()
    ac = compile_circuit(circ, order_trials=8)
    t_compile = time.perf_counter() - t0
    g5 = ACGraph(ac, device=0)
    th5 = torch.tensor([[0.30, 0.25, 0.50, 0.20], [1.20, 0.90, 0.40, 0.60]], dtype=torch.float64, device=dev)
    g5.sample(th5, 4096, 1, 1, 1, 1, dtype="c64", validate=False)
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record()
    g5.sample(th5, 4096, 1, 10, 1, 2, dtype="c64", validate=False)
    b.record()
    torch.cuda.synchronize()
    t5 = a.elapsed_time(b) / 1e3
    out.update({"qaoa_n32_p2_ac_nodes": g5.info["n_internal"], "qaoa_n32_p2_compile_s": t_compile,
                "qaoa_n32_p2_chains": 8192, "qaoa_n32_p2_sample_ms": t5 * 1e3,
                "qaoa_n32_p2_samples_per_s": 8192 / t5})
    g5.release_workspaces()
    g5.close()
    return out


def vqe_leg(steps: int):
    """The 2D Ising VQE workload on the same kernels: a noise-free 5x5 grid
    with one iteration (25 qubits) and a 3x3 grid with two iterations under
    depolarizing noise 0.005 after every gate; 256 parameter sets x 1000
    Gibbs samples each, complex64, 10 burn-in sweeps; Ising energy of every
    sample from the output bits."""
    import numpy as np
    import torch

    import workloads as W
    from paper_2103_17226_amd.api import ACGraph
    out = {}
    for tag, (rows, cols, p, dep) in {"ideal_5x5_p1": (5, 5, 1, None), "noisy_3x3_p2": (3, 3, 2, 0.005)}.items():
        _, J, h = W.ising_instance(rows, cols, W.sub_seed("graph", 6))
        circ = W.vqe_ising(rows, cols, p, J, h, dep=dep)
        g = ACGraph(circ, device=0)
        theta = torch.as_tensor(W.uniform_angles(256, circ.n_angles, W.sub_seed("angles", 6)), device=g.torch_device)
        C = 1000
        g.sample(theta, C, 1, 10, 1, 3, dtype="c64", validate=False)
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        for k in range(steps):
            res = g.sample(theta, C, 1, 10, 1, 4 + k, dtype="c64", want_rounds=True, validate=False)
        b.record()
        torch.cuda.synchronize()
        t = a.elapsed_time(b) / steps / 1e3
        x = res["samples"].cpu().numpy().reshape(-1).view(np.uint64)
        bits = ((x[:, None] >> np.arange(circ.n, dtype=np.uint64)) & np.uint64(1)).astype(np.int64)
        e = W.ising_energy(circ.edges, J, h, bits).reshape(256, C).mean(axis=1)
        out[tag] = {"qubits": circ.n, "iterations": p, "gates": circ.n_gates(),
                    "ac_internal_nodes": g.info["n_internal"], "ac_edges": g.info["n_edges"],
                    "samples_per_s": 256 * C / t, "ms_per_256k_samples": t * 1e3,
                    "gibbs_rounds_per_sample": float(res["rounds"].double().mean().item()),
                    "best_mean_energy": float(e.min())}
        g.close()
    return out


def cpu_baseline(circ, theta, chains, budget_s):
    """The oracle on the host cores, on a bounded sample of the same job:
    per parameter set, the density-matrix diagonal, `chains` exact samples by
    inverse CDF, and the parameter-shift gradient of <C>."""
    import numpy as np
    import torch
    from oracle import grad as ograd
    from oracle import sim
    rng = np.random.default_rng(0)
    done = 0
    t0 = time.perf_counter()
    while done < theta.shape[0]:
        th = theta[done]
        p = sim.probabilities(circ, th)
        p = p / p.sum()
        cdf = np.cumsum(p)
        _ = np.searchsorted(cdf, rng.random(chains) * cdf[-1], side="right")
        _ = ograd.expected_cost_param_shift(circ, th)
        done += 1
        if time.perf_counter() - t0 > budget_s:
            break
    dt = time.perf_counter() - t0
    try:                                   # threads of the BLAS the oracle's matrix products use
        from threadpoolctl import threadpool_info
        cores = max([int(i.get("num_threads", 1)) for i in threadpool_info() if i.get("user_api") == "blas"] or [1])
    except Exception:
        cores = torch.get_num_threads()
    return {"value": done * chains / dt, "unit": "samples/s", "cores": cores,
            "kind": "oracle",
            "sample": f"{done} of {theta.shape[0]} parameter sets: density-matrix diagonal, {chains} "
                      f"exact samples each, parameter-shift gradient of <C> ({dt:.1f} s, numpy complex128)",
            "host": host_description()}


def host_description():
    """CPU model and logical core count of the host."""
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"cpu_model": model, "os_cpu_count": os.cpu_count(),
            "usable_cores": len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()}


def cpu_evaluator_baseline(circ, theta, chains, eval_cfg, budget_s, method, order_trials):
    """The plain CPU AC evaluator (libqkc_cpu.so, complex128, OpenMP) on
    the same blobs: Gibbs samples/s on the default sampling job's AC (a
    bounded slice of its parameter sets, all chains each) and upward-pass
    node-evals/s on the 16-qubit amplitude job's rows, on all usable cores
    and on one core."""
    import numpy as np

    from paper_2103_17226_amd import cpu_eval
    from paper_2103_17226_amd.blob import to_blob
    cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    out = {"kind": "plain CPU AC evaluator (C++ -O3, OpenMP, complex128; same blobs, same sampler rules)",
           "host": host_description()}
    sac = cpu_eval.CpuAC(to_blob(compile_ac(circ, method, order_trials)))
    eac = cpu_eval.CpuAC(to_blob(compile_ac(eval_cfg["circuit"], method)))
    for label, threads in (("all_cores", cores), ("one_core", 1)):
        share = budget_s / 4.0
        # samples: parameter sets one after another, all their chains, until the time share is used
        done, t0 = 0, time.perf_counter()
        while done < theta.shape[0] and time.perf_counter() - t0 < share:
            step = max(1, min(theta.shape[0] - done, threads // 8 or 1))
            sac.sample(theta[done:done + step], chains, 1, 10, 1, seed=7, threads=threads)
            done += step
        ts = time.perf_counter() - t0
        # amplitudes: blocks of 4096 rows of the 16-qubit job
        ev, po, th = eval_cfg["evidence"], eval_cfg["param_of"], eval_cfg["theta"]
        rows, t0 = 0, time.perf_counter()
        while rows < ev.shape[0] and time.perf_counter() - t0 < share:
            blk = 4096 if threads > 1 else 256
            sl = slice(rows, rows + blk)
            sac_amp = eac.eval(th, ev[sl], po[sl], threads=threads)
            rows += blk
        te = time.perf_counter() - t0
        out[label] = {"threads": threads, "samples_per_s": done * chains / ts,
                      "sample_job": f"{done} parameter sets x {chains} chains, 10 burn-in sweeps ({ts:.1f} s)",
                      "node_evals_per_s": rows * eac.n_internal / te, "amplitudes_per_s": rows / te,
                      "eval_job": f"{rows} rows of the 16-qubit p=2 batch ({te:.1f} s)"}
        del sac_amp
    return out


def main():
    args = parse()
    if args.copy_probe:
        copy_probe()
        return
    if args.gpus != 1:
        print(json.dumps({"error": "the library runs on one GPU; --gpus must be 1",
                          "n_gpus_requested": args.gpus}))
        sys.exit(2)
    pool = blobs = None
    t_pool = 0.0
    started = None
    if not args.no_serve:         # compiles while the GPU legs run
        started = compile_pool_start(args.serve_pool == "full", args.blob_cache)
        if not 1 <= args.serve_hw_queues <= 32:
            sys.exit("--serve-hw-queues must be in [1, 32]")
        os.environ["GPU_MAX_HW_QUEUES"] = str(args.serve_hw_queues)     # before HIP starts
    import numpy as np
    import torch

    import workloads as W
    from paper_2103_17226_amd import _lib
    from paper_2103_17226_amd.api import ACGraph

    if not torch.cuda.is_available():
        print(json.dumps({"error": "no HIP device"}))
        sys.exit(1)
    _lib.lib()
    dev = torch.device("cuda", 0)
    cfg = W.config(2)
    circ = cfg["circuit"]
    P, chains = args.params, args.chains
    theta_np = cfg["theta"][:P]
    g = ACGraph(compile_ac(circ, args.compiler, order_trials=args.order_trials), device=0)
    info = g.info
    theta = torch.as_tensor(theta_np, dtype=torch.float64, device=dev)
    edges = torch.as_tensor(np.asarray(circ.edges, dtype=np.int32), device=dev)
    S = chains
    param_of = torch.arange(P, dtype=torch.int32, device=dev).repeat_interleave(S)
    Wn = info["n_words"]
    ev_t = {}
    ws_sample = g.workspace(args.dtype, P * chains, _lib.AC_OP_SAMPLE)

    def step(seed):
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        ev2 = torch.cuda.Event(enable_timing=True)
        ev0.record()
        s = g.sample(theta, chains_per_param=chains, samples_per_chain=1, burn_in=args.burn_in, thin=1,
                     seed=seed, cost_edges=edges, dtype=args.dtype, want_states=True, want_cost=True,
                     want_rounds=True, validate=False, ws=ws_sample)
        ev1.record()
        out = g.grad(theta, s["states"].view(P * S, Wn), param_of, mode="logprob",
                     weight=s["cost"].view(P * S), dtype=args.dtype, validate=False)
        ev2.record()
        ev_t.setdefault("ev", []).append((ev0, ev1, ev2))
        return s, out

    for i in range(args.warmup):
        step(1000 + i)
    torch.cuda.synchronize()
    ev_t.clear()
    t0 = time.perf_counter()
    last = None
    for i in range(args.steps):
        last = step(2000 + i)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    dt = (t1 - t0) / args.steps
    samp_ms = [a.elapsed_time(b) for a, b, c in ev_t["ev"]]
    grad_ms = [b.elapsed_time(c) for a, b, c in ev_t["ev"]]
    s, out = last
    rounds = float(s["rounds"].double().sum().item())
    N, E = info["n_internal"], info["n_edges"]
    comp = g.compiled
    tags = comp.col >> 30
    E_ii = int((tags == 0).sum())
    n_ind = info["n_indicator_leaves"]
    cs = 8 if args.dtype == "c64" else 16
    # algorithmic bytes per chain-round: the streaming model on the
    # sum-of-products plan the sampler runs (every super-node value written
    # once and every super-node factor read once in the upward pass; the
    # downward pass reads the parent adjoint and sibling rows of every
    # occurrence and writes each adjoint; the leaf step reads the same for
    # indicator and selector occurrences and writes one derivative per
    # variable value; the evidence words once)
    p_up, p_down, p_leaf = plan_byte_model(info, cs)
    bytes_round = (p_up - cs) + p_down + p_leaf
    # the same model on the compiled DAG (every node a row), for comparison
    dag_bytes_round = cs * (E_ii + N) + cs * (N + 2 * E_ii) + cs * n_ind + 8 * Wn
    samp_s = float(np.mean(samp_ms)) / 1e3
    achieved = bytes_round * rounds / samp_s / 1e9
    default_run = (P, chains, args.burn_in, args.dtype, args.order_trials) == (1024, 1000, 10, "c64", 64)
    node_evals = 2.0 * N * rounds + 2.0 * N * P * S
    samples = P * S
    res = {
        "metric": METRIC,
        "value": samples / dt,
        "unit": "samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.dtype,
        "data": "synthetic",
        "config": {
            "workload": "noisy QAOA p=1 MaxCut, seeded random 3-regular graph, 8 qubits, depolarizing "
                        "p=0.01 after every gate; 1024 (gamma,beta) sets x 1000 Gibbs samples + "
                        "score-function gradient of <C> over the samples",
            "param_sets": P, "samples_per_param": S, "burn_in_sweeps": args.burn_in,
            "ac_internal_nodes": N, "ac_edges": E, "ac_levels": info["n_levels"],
            "evidence_vars": info["n_vars"], "ac_compiler": args.compiler,
        },
        "node_evals_per_s": node_evals / dt,
        "amplitude_node_evals_per_s_sampler": 2.0 * N * rounds / samp_s,
        "gibbs_rounds_per_sample": rounds / samples,
        "sampler_ms": float(np.mean(samp_ms)),
        "grad_ms": float(np.mean(grad_ms)),
        "roofline": {
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": profiled_traffic("k_sample_stream", default_run, g.blob),
            "kernel_sha256_16": kernel_sha16(), "ac_sha256_16": _sha16(g.blob),
            "traffic_unit": "HBM bytes per dispatch (rocprofv3)",
            "kernel": "k_sample_stream (Gibbs rounds: upward + downward pass + decisions; "
                      "timed with HIP events around ac_sample on its stream)",
            "bytes_per_chain_round": bytes_round,
            "ac_super_nodes": info["n_super"],
            "dag_model_bytes_per_chain_round": dag_bytes_round,
            "dag_model_GBps": dag_bytes_round * rounds / samp_s / 1e9,
        },
    }
    del s, out, last
    g.close()
    ws_sample = None
    torch.cuda.empty_cache()
    copy_gbs = copy_peak_gbs(dev)
    res["roofline"]["copy_peak_GBps"] = copy_gbs
    res["roofline"]["frac_of_copy_peak"] = achieved / copy_gbs
    if not args.no_eval:
        print("# amplitude/gradient leg (16 qubits, p=2)", file=sys.stderr, flush=True)
        res["eval"] = eval_leg(args, W.config(3))
        res["eval"]["roofline"]["frac_of_copy_peak"] = res["eval"]["roofline"]["achieved"] / copy_gbs
        print("# 4-qubit ring and 32-qubit sampling", file=sys.stderr, flush=True)
        res["other_configs"] = small_configs_leg(args.eval_steps)
        print("# 2D Ising VQE", file=sys.stderr, flush=True)
        res["vqe"] = vqe_leg(args.eval_steps)
        print("# most probable explanations", file=sys.stderr, flush=True)
        res["mpe"] = mpe_leg(args.eval_steps, args.mpe_params)
        torch.cuda.empty_cache()
    if started is not None:
        print("# serving pool (compiled in the background)", file=sys.stderr, flush=True)
        pool, blobs, t_pool, cache_hits = compile_pool_finish(started)
        graphs = {c.name: ACGraph(b, device=0) for c, b in zip(pool, blobs)}
        print("# admission estimate, requests alone", file=sys.stderr, flush=True)
        est_alone = estimate_check(graphs, pool, args)
        runs = []
        for rate in [float(x) for x in args.serve_rates.split(",") if x]:
            print(f"# serving at {rate:g} req/s", file=sys.stderr, flush=True)
            runs.append(serve_run(graphs, pool, rate, args))
        res["serving"] = {
            "workload": "serving mix: noisy QAOA p in {1,2}, n in {6,8,12,16,20}, 4 graphs each, "
                        "Poisson arrivals; P~logU{1..256}, eval(64 x/set) w.p. 0.1 else S~logU{1..4096} "
                        "samples/set (S>=2 with a gradient), gradient w.p. 0.5; c64",
            "pool_circuits": len(pool), "pool_compile_s": t_pool, "pool_cache_hits": cache_hits,
            "pool_ac_nodes_max": max(gr.info["n_internal"] for gr in graphs.values()),
            "streams": args.serve_streams, "hw_queues": os.environ.get("GPU_MAX_HW_QUEUES"),
            "queue_limit": args.serve_queue,
            "budget_gib": args.serve_budget_gib, "max_request_seconds": args.serve_max_seconds,
            "part_streams": args.serve_part_streams, "part_share": args.serve_part_share,
            "max_split": args.serve_max_split, "split_backlog_s": args.serve_split_backlog,
            "warmup_s": args.serve_warmup, "measured_s": args.serve_seconds,
            "measured_s_lower_rates": args.serve_seconds_low,
            "estimate_alone": est_alone,
            "runs": runs,
        }
        main_run = max(runs, key=lambda r: r["offered_rps"]) if runs else {}
        res["serving"]["p50_ms"] = main_run.get("p50_ms")
        res["serving"]["p99_ms"] = main_run.get("p99_ms")
        for gr in graphs.values():
            gr.close()
        torch.cuda.empty_cache()
    if not args.no_cpu_baseline:    # last: the host cores are idle by now
        print("# CPU baselines", file=sys.stderr, flush=True)
        res["cpu_baseline"] = cpu_baseline(circ, theta_np, chains, args.cpu_seconds)
        res["cpu_evaluator"] = cpu_evaluator_baseline(circ, theta_np, chains, W.config(3), args.cpu_seconds,
                                                      args.compiler, args.order_trials)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
