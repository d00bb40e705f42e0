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

Prints one JSON line.  --gpus > 1 is refused: this build runs on one GPU.
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


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--burn-in", type=int, default=10)
    ap.add_argument("--params", type=int, default=1024)
    ap.add_argument("--chains", type=int, default=1000)
    ap.add_argument("--dtype", default="c64")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--copy-probe", action="store_true",
                    help="only copy 1 GiB device-to-device three times (calibrates the HBM "
                         "byte counters of a profiler run) and exit")
    return ap.parse_args()


def copy_probe():
    import torch
    a = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes": 3 * (1 << 30)}))


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
    return {"value": done * chains / dt, "unit": "samples/s", "cores": torch.get_num_threads(),
            "kind": "oracle",
            "sample": f"{done} of {theta.shape[0]} parameter sets: density-matrix diagonal, {chains} "
                      f"exact samples each, parameter-shift gradient of <C> ({dt:.1f} s, numpy complex128)"}


def main():
    args = parse()
    if args.copy_probe:
        copy_probe()
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1",
                          "n_gpus_requested": args.gpus}))
        sys.exit(2)
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
    g = ACGraph(circ, device=0)
    info = g.info
    theta = torch.as_tensor(theta_np, dtype=torch.float64, device=dev)
    edges = torch.as_tensor(np.asarray(circ.edges, dtype=np.int32), device=dev)
    S = chains
    param_of = torch.arange(P, dtype=torch.int32, device=dev).repeat_interleave(S)
    Wn = info["n_words"]
    ev_t = {}

    def step(seed):
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        ev2 = torch.cuda.Event(enable_timing=True)
        ev0.record()
        s = g.sample(theta, chains_per_param=chains, samples_per_chain=1, burn_in=args.burn_in, thin=1,
                     seed=seed, cost_edges=edges, dtype=args.dtype, want_states=True, want_cost=True,
                     want_rounds=True, validate=False)
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
    # algorithmic bytes per chain-round (streaming model: every node value
    # written once and every internal child read once in the upward pass;
    # the downward pass reads the node values and parent adjoints and writes
    # each adjoint; one indicator derivative per variable value)
    bytes_round = cs * (E_ii + N) + cs * (N + 2 * E_ii) + cs * n_ind + 8 * Wn
    samp_s = float(np.mean(samp_ms)) / 1e3
    achieved = bytes_round * rounds / samp_s / 1e9
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
            "evidence_vars": info["n_vars"],
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
            "traffic": None,
            "kernel": "k_sample (Gibbs: upward + downward pass + decisions)",
            "bytes_per_chain_round": bytes_round,
        },
    }
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline(circ, theta_np, chains, args.cpu_seconds)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
