"""Served results equal the plain calls: every request of a mixed stream
(amplitudes, gradients, samples, sampled gradients over several resident
graphs) gets, through the continuous-batching loop with merged launches and
overlapping streams, what the same request gets from the plain binding calls
on its own.  Amplitudes and samples are compared bit for bit, gradients to
1e-12 relative (the merged reduction is arranged to add the same terms in the
same order, so they are expected to agree bit for bit too)."""
import time

import numpy as np
import pytest
import torch

import workloads as W
from tests.gpu_common import graph, note, oracle_amplitudes, require_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _gpu():
    require_gpu()


def _pool():
    pool = W.serving_pool()
    pick = [pool[0], pool[4], pool[20]]          # n=6 p=1, n=8 p=1, n=6 p=2
    return {c.name: c for c in pick}


def _requests(circs, n, seed):
    names = sorted(circs)
    pool = [circs[k] for k in names]
    raw = W.serving_requests(pool, rate=200.0, duration=2.0 * n / 200.0, seed=seed, max_params=12, max_samples=96,
                             p_eval=0.5)[:n]
    return [(names[r["circuit"]], r) for r in raw]


def _plain(g, circ, r, dtype="c64"):
    """The request through the plain binding calls, on its own."""
    theta = r["theta"]
    out = {}
    if r["samples"] == 0:
        if r["grad"]:
            res = g.grad(theta, r["evidence"], r["param_of"], mode="prob", weight=r["weight"], dtype=dtype,
                         want_amp=True)
            out = {"amp": res["amp"].cpu().numpy(), "grad": res["grad"].cpu().numpy()}
        else:
            amp, prob = g.eval(theta, r["evidence"], r["param_of"], dtype=dtype)
            out = {"amp": amp.cpu().numpy(), "prob": prob.cpu().numpy()}
        return out
    S, P = r["samples"], theta.shape[0]
    res = g.sample(theta, chains_per_param=S, samples_per_chain=1, burn_in=10, thin=1, seed=r["seed"],
                   cost_edges=circ.edges, dtype=dtype, want_cost=True, want_states=r["grad"])
    out = {"samples": res["samples"].cpu().numpy(), "cost": res["cost"].cpu().numpy()}
    if r["grad"]:
        from paper_2103_17226_amd.serve import loo_score_gradient
        cost = res["cost"]
        po = torch.arange(P, dtype=torch.int32, device=cost.device).repeat_interleave(S)
        st = res["states"].reshape(P * S, -1)
        A = g.grad(theta, st, po, mode="logprob", weight=cost.reshape(-1), dtype=dtype)["grad"].cpu().numpy()
        G = g.grad(theta, st, po, mode="logprob", weight=np.ones(P * S), dtype=dtype)["grad"].cpu().numpy()
        out["grad"] = loo_score_gradient(A, G, out["cost"].sum(axis=1), S)
    return out


def _request(name, r):
    from paper_2103_17226_amd.serve import Request
    return Request(graph=name, theta=r["theta"], evidence=r.get("evidence"), param_of=r.get("param_of"),
                   weight=r.get("weight"), samples=r["samples"], grad=r["grad"], burn_in=10, seed=r["seed"])


def _same(served, plain, what):
    assert set(served) == set(plain), what
    for k in plain:
        a, b = np.asarray(served[k]), np.asarray(plain[k])
        assert a.shape == b.shape, (what, k)
        if k == "grad":
            scale = max(np.max(np.abs(b)), 1e-30)
            assert np.max(np.abs(a - b)) <= 1e-12 * scale, (what, k, np.max(np.abs(a - b)) / scale)
        else:
            assert np.array_equal(a.view(np.uint8), b.view(np.uint8)), (what, k)


def test_split_requests_equal_the_whole_request():
    # With a small device-time limit, large requests are split into parts
    # (parameter sets, or chains / rows of one set) that flow through the
    # loop; each reassembled result equals the whole request through the
    # plain binding calls: samples and costs bit for bit (the parts' chain
    # offsets draw the same chains), amplitudes bit for bit, gradients to
    # 1e-12 of their largest entry.
    from paper_2103_17226_amd.serve import GraphExecutor, Server
    circs = _pool()
    graphs = {k: graph(c) for k, c in circs.items()}
    names = sorted(circs)
    raw = W.serving_requests([circs[k] for k in names], rate=200.0, duration=1.0, seed=91, max_params=48,
                             max_samples=1500, p_eval=0.25)[:24]
    reqs = [(names[r["circuit"]], r) for r in raw if not (r["samples"] == 1 and r["grad"])]
    plain = [_plain(graphs[k], circs[k], r) for k, r in reqs]
    torch.cuda.synchronize()
    ex = GraphExecutor(graphs, {k: c.edges for k, c in circs.items()}, n_streams=4)

    def smallest_part(k, r):            # one chain, or one evidence row, of one parameter set
        q = _request(k, r)
        q.theta = np.asarray(q.theta)[:1]
        if q.kind == "sample":
            q.samples = 1
        else:
            q.evidence, q.param_of = q.evidence[:1], np.zeros(1, np.int32)
            q.weight = None if q.weight is None else q.weight[:1]
        return ex.cost(q)
    limit = 1.05 * max(smallest_part(k, r) for k, r in reqs)     # every request can be split to fit
    n_over = sum(ex.cost(_request(k, r)) > limit for k, r in reqs)
    note(f"serve split: limit {limit:.3g} s, {n_over} of {len(reqs)} requests over it")
    assert n_over >= 1
    srv = Server(ex, mem_budget=8 << 30, max_merge=16, max_seconds=limit, max_split=len(reqs),
                 split_backlog=float("inf"), part_streams=2, part_share=0.5)
    futs = [srv.submit(_request(k, r)) for k, r in reqs]
    srv.start()
    try:
        results = [f.result(timeout=300) for f in futs]
    finally:
        srv.stop()
    st = srv.latency_stats()
    note(f"serve split: {st}")
    assert st["completed"] == len(reqs) and st["rejected_cost"] == 0 and st["split_requests"] == n_over
    for i, ((k, r), got, want) in enumerate(zip(reqs, results, plain)):
        _same(got, want, f"request {i} on {k} (samples={r['samples']}, grad={r['grad']})")


def test_sweep_slices_resume_the_same_chains():
    # a limit below one chain's full run: sampling requests are cut into
    # slices of their sweeps, each resuming the chain states the slice before
    # it left on the device; samples, costs and sampled gradients equal the
    # whole request's
    from paper_2103_17226_amd.serve import GraphExecutor, Request, Server
    circs = _pool()
    name = sorted(circs)[2]
    circ = circs[name]
    g = graph(circ)
    ex = GraphExecutor({name: g}, {name: circ.edges}, n_streams=3)
    rng = np.random.default_rng(31)
    reqs = [dict(theta=rng.uniform(0, 2 * np.pi, size=(P, circ.n_angles)), samples=S, grad=gr, seed=s,
                 evidence=None, param_of=None, weight=None)
            for P, S, gr, s in ((2, 300, True, 5), (1, 700, False, 6), (3, 64, True, 7))]
    plain = [_plain(g, circ, r) for r in reqs]
    torch.cuda.synchronize()
    one_sweep = ex.cost(Request(graph=name, theta=reqs[0]["theta"][:1], samples=1, burn_in=0))
    limit = 2.5 * one_sweep
    srv = Server(ex, mem_budget=8 << 30, max_seconds=limit, max_split=8, split_backlog=float("inf"),
                 part_streams=2, part_share=0.5)
    qs = [_request(name, r) for r in reqs]
    for q in qs:
        parts = ex.split(q, limit)
        assert parts and any(u.part[5] > 0 for u in parts), "no sweep slices"
    futs = [srv.submit(q) for q in qs]
    srv.start()
    try:
        results = [f.result(timeout=300) for f in futs]
    finally:
        srv.stop()
    st = srv.latency_stats()
    note(f"serve sweep slices: limit {limit:.3g} s, {st['split_parts']} parts")
    assert st["completed"] == len(reqs) and not ex._carry
    for i, (got, want) in enumerate(zip(results, plain)):
        _same(got, want, f"request {i}")


def test_served_equals_alone_in_a_mixed_stream():
    from paper_2103_17226_amd.serve import GraphExecutor, Server
    circs = _pool()
    note("serve: compile and load 3 graphs")
    graphs = {k: graph(c) for k, c in circs.items()}
    reqs = [(k, r) for k, r in _requests(circs, 64, seed=77) if not (r["samples"] == 1 and r["grad"])][:60]
    kinds = {(r["samples"] > 0, r["grad"]) for _, r in reqs}
    assert len(kinds) == 4, kinds
    note(f"serve: plain calls for {len(reqs)} requests")
    plain = [_plain(graphs[k], circs[k], r) for k, r in reqs]
    torch.cuda.synchronize()
    note("serve: the same requests through the loop (4 streams, merging)")
    ex = GraphExecutor(graphs, {k: c.edges for k, c in circs.items()}, n_streams=4)
    srv = Server(ex, mem_budget=8 << 30, max_merge=16)
    futs = [srv.submit(_request(k, r)) for k, r in reqs]      # queued before the loop starts: merges
    srv.start()
    try:
        results = [f.result(timeout=120) for f in futs]
    finally:
        srv.stop()
    st = srv.latency_stats()
    note(f"serve: {st}")
    assert st["completed"] == len(reqs) and st["failed"] == 0
    assert st["merged"] > 0 and st["max_inflight"] > 1
    for i, ((k, r), got, want) in enumerate(zip(reqs, results, plain)):
        _same(got, want, f"request {i} on {k} (samples={r['samples']}, grad={r['grad']})")


def test_served_amplitudes_match_the_oracle():
    from paper_2103_17226_amd.serve import GraphExecutor, Request, Server
    circs = _pool()
    name = sorted(circs)[0]
    circ = circs[name]
    note(f"serve vs oracle on {name}")
    g = graph(circ)
    rng = np.random.default_rng(5)
    ex = GraphExecutor({name: g}, n_streams=2)
    srv = Server(ex, mem_budget=1 << 30)
    srv.start()
    try:
        out = _submit_oracle_batch(srv, name, circ, rng, inputs := [])
    finally:
        srv.stop()
    for (theta, vals, po), res in zip(inputs, out):
        ref = np.array([oracle_amplitudes(circ, theta[po[b]], vals[b:b + 1])[0] for b in range(len(po))])
        assert np.max(np.abs(res["amp"] - ref)) <= 1e-12
        np.testing.assert_allclose(res["prob"], np.abs(ref) ** 2, rtol=1e-10, atol=1e-15)


def _submit_oracle_batch(srv, name, circ, rng, inputs):
    from paper_2103_17226_amd.serve import Request
    futs = []
    for i in range(6):
        P, B = 1 + i, 10 + 7 * i
        theta = rng.uniform(0, 2 * np.pi, size=(P, circ.n_angles))
        vals = np.zeros((B, circ.n_vars), dtype=np.int64)
        vals[:, :circ.n] = rng.integers(0, 2, size=(B, circ.n))
        doms = circ.var_domains()
        for v in range(circ.n, circ.n_vars):
            vals[:, v] = rng.integers(0, doms[v], size=B) * (rng.random(B) < 0.1)
        po = rng.integers(0, P, size=B).astype(np.int32)
        inputs.append((theta, vals, po))
        futs.append(srv.submit(Request(graph=name, theta=theta, evidence=W.pack_evidence(circ, vals),
                                       param_of=po, dtype="c128")))
    return [f.result(timeout=60) for f in futs]


def test_loop_admits_while_others_run_and_reports_latency():
    from paper_2103_17226_amd.serve import GraphExecutor, Server
    circs = _pool()
    graphs = {k: graph(c) for k, c in circs.items()}
    reqs = [(k, r) for k, r in _requests(circs, 44, seed=91) if not (r["samples"] == 1 and r["grad"])][:40]
    note("serve: timed arrivals")
    ex = GraphExecutor(graphs, {k: c.edges for k, c in circs.items()}, n_streams=4)
    srv = Server(ex, mem_budget=8 << 30)
    srv.start()
    try:
        t0 = time.perf_counter()
        futs = []
        for k, r in reqs:
            delay = t0 + r["t"] - time.perf_counter()
            if delay > 0:
                time.sleep(delay)
            futs.append(srv.submit(_request(k, r)))
        for f in futs:
            f.result(timeout=120)
    finally:
        srv.stop()
    st = srv.latency_stats()
    note(f"serve: {st}")
    assert st["completed"] == len(reqs)
    assert 0 < st["p50_ms"] <= st["p99_ms"]
    # some request started before an earlier one had finished: launches overlapped
    done = sorted(srv.completed, key=lambda r: r.t_start)
    assert any(b.t_start < a.t_done for a, b in zip(done, done[1:]))


def test_session_resumes_its_resident_chains():
    from paper_2103_17226_amd.serve import GraphExecutor, Request, Server
    circs = _pool()
    name = sorted(circs)[1]
    circ = circs[name]
    note(f"serve: session chains on {name}")
    g = graph(circ)
    rng = np.random.default_rng(12)
    th1 = rng.uniform(0, 2 * np.pi, size=(2, circ.n_angles))
    th2 = th1 + 0.05                                   # the optimiser's next iterate
    ex = GraphExecutor({name: g}, {name: circ.edges}, n_streams=2)
    srv = Server(ex, mem_budget=1 << 30)
    srv.start()
    try:
        f1 = srv.submit(Request(graph=name, theta=th1, samples=50, burn_in=5, seed=9, session="opt"))
        f2 = srv.submit(Request(graph=name, theta=th2, samples=50, burn_in=0, seed=9, session="opt"))
        r1, r2 = f1.result(timeout=60), f2.result(timeout=60)
        assert ex.resident_bytes() == 2 * 50 * g.info["n_words"] * 8
        srv.close_session(name, "opt")
    finally:
        srv.stop()
    assert ex.resident_bytes() == 0
    p1 = g.sample(th1, 50, 1, 5, 1, 9, cost_edges=circ.edges, want_cost=True, want_states=True)
    p2 = g.sample(th2, 50, 1, 0, 1, 9, cost_edges=circ.edges, want_cost=True,
                  init_states=p1["states"].reshape(100, -1), first_sweep=6)
    assert np.array_equal(r1["samples"], p1["samples"].cpu().numpy())
    assert np.array_equal(r2["samples"], p2["samples"].cpu().numpy())
    assert np.array_equal(r2["cost"], p2["cost"].cpu().numpy())


def test_sample_shape_reports_the_kernel_sample_runs(monkeypatch):
    """ac_sample_shape (used by the serving cost model) names the kernel
    ac_sample picks and how many chains it advances at once."""
    note("sampler shape query")
    g = graph(W.config(2, small=True)["circuit"])
    kind, conc = g.sample_shape("c64", 64)
    assert kind == "lds" and 1 <= conc <= 64
    kind, conc = g.sample_shape("c64", 1_024_000)
    assert kind == "stream" and conc % 64 == 0 and 64 <= conc < 1_024_000
    assert g.sample_shape("c128", 1_024_000)[0] == "stream"
    for forced in ("global", "stream", "lds"):
        monkeypatch.setenv("QKC_SAMPLE_KERNEL", forced)
        assert g.sample_shape("c64", 4096)[0] == forced
    monkeypatch.delenv("QKC_SAMPLE_KERNEL")
    with pytest.raises(Exception):
        g.sample_shape("c64", 0)
