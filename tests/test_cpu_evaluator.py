"""The plain CPU evaluator (libqkc_cpu.so, the timing baseline) against the
oracle, on the CPU: amplitudes of every op kind and channel in complex128,
derivative-driven Gibbs chains decision for decision against the oracle's
reference chain, and the exported symbols of include/qkc_cpu.h."""
import os
import re

import numpy as np
import pytest

import workloads as W
from oracle import gibbs, sim
from paper_2103_17226_amd import cpu_eval
from paper_2103_17226_amd.blob import to_blob
from paper_2103_17226_amd.compiler import compile_circuit

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_library_exports_every_declared_symbol():
    txt = open(os.path.join(ROOT, "include", "qkc_cpu.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    declared = sorted(set(re.findall(r"\b(qkc_cpu_[a-z_]+)\s*\(", txt)))
    assert declared == sorted(cpu_eval.EXPORTED)
    lib = cpu_eval.lib()
    for name in declared:
        assert hasattr(lib, name), name


def _values(circ, B, rng):
    return np.concatenate([rng.integers(0, 2, size=(B, circ.n)), W.sample_channel_prior(circ, B, rng)], axis=1)


@pytest.mark.parametrize("seed", [1, 2, 3, 4])
def test_amplitudes_match_the_oracle_on_random_circuits(seed):
    circ = W.random_circuit(seed)
    ac = cpu_eval.CpuAC(to_blob(compile_circuit(circ)))
    rng = np.random.default_rng(seed)
    P, B = 3, 60
    theta = rng.uniform(-3, 3, size=(P, circ.n_angles))
    vals = np.concatenate([rng.integers(0, 2, size=(B, circ.n)),
                           np.stack([rng.integers(0, d, size=B) for d in circ.var_domains()[circ.n:]], axis=1)
                           if circ.n_vars > circ.n else np.zeros((B, 0), np.int64)], axis=1)
    po = (np.arange(B) % P).astype(np.int32)
    amp = ac.eval(theta, W.pack_evidence(circ, vals), po, threads=2)
    for b in range(B):
        x = sum(int(vals[b, q]) << q for q in range(circ.n))
        ref = sim.amplitude(circ, theta[po[b]], x, vals[b, circ.n:])
        assert abs(amp[b] - ref) <= 1e-12, (b, amp[b], ref)


def test_amplitudes_of_config3_rows_and_a_noise_override():
    cfg = W.config(3, small=True)
    circ = cfg["circuit"]
    ac = cpu_eval.CpuAC(to_blob(compile_circuit(circ)))
    ev, po, th = cfg["evidence"][:24], cfg["param_of"][:24], cfg["theta"]
    vals = W.unpack_evidence(circ, ev)
    noise = np.array(circ.noise) * 1.7
    for nz in (None, noise):
        amp = ac.eval(th, ev, po, noise=nz)
        for b in range(0, 24, 5):
            x = sum(int(vals[b, q]) << q for q in range(circ.n))
            ref = sim.amplitude(circ, th[po[b]], x, vals[b, circ.n:], noise=nz)
            assert abs(amp[b] - ref) <= 1e-12


def test_chains_follow_the_oracle_chain():
    circ = W.qaoa_maxcut(3, W.ring_graph(3), 1, dep=0.05, ad=0.03)
    ac = cpu_eval.CpuAC(to_blob(compile_circuit(circ)))
    theta = np.array([[0.7, 0.4], [2.1, 1.2]])
    C, burn, thin, S = 5, 3, 2, 2
    out = ac.sample(theta, C, S, burn, thin, seed=17, want_states=True, threads=3)
    got = W.unpack_evidence(circ, out["states"].reshape(-1, ac.n_words))
    for p in range(2):
        for c in range(C):
            ref, _ = gibbs.run_chain(circ, theta[p], seed=17, chain=p * C + c, burn_in=burn, thin=thin,
                                     n_samples=S)
            i = p * C * S + c * S
            assert np.array_equal(got[i:i + S], ref), (p, c)
            # one pass per change of state, plus one after the last change
            bc = gibbs.BranchCache(circ, theta[p])
            s = gibbs.init_state(circ, 17, p * C + c)
            changes, last = 0, False
            for sw in range(burn + S * thin):
                for v in range(circ.n_vars):
                    u = gibbs.choose(gibbs.conditional_weights(bc, s, v), gibbs.uniform(17, p * C + c, sw, v))
                    last = u is not None and u != s[v]
                    if last:
                        s[v], changes = u, changes + 1
            assert out["rounds"].reshape(-1)[p * C + c] == changes + (0 if last else 1)


def test_results_do_not_depend_on_the_thread_count():
    cfg = W.config(2, small=True)
    ac = cpu_eval.CpuAC(to_blob(compile_circuit(cfg["circuit"])))
    a = ac.sample(cfg["theta"][:4], 16, seed=3, threads=1)
    b = ac.sample(cfg["theta"][:4], 16, seed=3, threads=4)
    assert np.array_equal(a["samples"], b["samples"]) and np.array_equal(a["rounds"], b["rounds"])


def test_corrupt_blobs_are_refused():
    blob = to_blob(compile_circuit(W.config(1, small=True)["circuit"]))
    with pytest.raises(RuntimeError, match="magic"):
        cpu_eval.CpuAC(b"X" + blob[1:])
    with pytest.raises(RuntimeError):
        cpu_eval.CpuAC(blob[:len(blob) // 2])
