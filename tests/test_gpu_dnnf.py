"""GPU parity of ACs from the search-based compiler (decision-DNNF read as an
AC): the library runs them through the same C ABI, and amplitudes, d f /
d theta and complex64 probabilities must meet the oracle as those of the
variable-elimination compiler do."""
import numpy as np
import pytest

import workloads as W
from oracle import grad as ograd
from oracle import sim
from paper_2103_17226_amd.dnnf import compile_circuit_dpll
from tests.gpu_common import graph, note, prob_ok, require_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _gpu():
    require_gpu()


@pytest.mark.parametrize("seed", range(6))
def test_dpll_random_circuits_on_the_gpu(seed):
    circ = W.random_circuit(seed)
    g = graph(compile_circuit_dpll(circ))
    note(f"dpll random circuit {seed}: {g.info['n_internal']} nodes, {g.info['n_super']} super-nodes")
    rng = np.random.default_rng(300 + seed)
    theta = rng.uniform(0, 2 * np.pi, size=(2, circ.n_angles))
    B = 64 * 2 + 9
    doms = circ.var_domains()
    vals = np.array([[int(rng.integers(0, d)) for d in doms] for _ in range(B)], dtype=np.int64)
    po = rng.integers(0, 2, size=B).astype(np.int32)
    ev = W.pack_evidence(circ, vals)
    out = g.grad(theta, ev, po, mode="cotangent", cotangent=np.ones(B, complex), dtype="c128", want_amp=True,
                 want_dfdtheta=True)
    amp = out["amp"].cpu().numpy()
    dft = out["dfdtheta"].cpu().numpy()
    ref = np.zeros(B, complex)
    cache = {}
    for b in range(B):
        p, k = int(po[b]), tuple(int(z) for z in vals[b, circ.n:])
        if (p, k) not in cache:
            kk = np.array(k, dtype=np.int64)
            cache[(p, k)] = (sim.branch_state(circ, theta[p], kk), ograd.amplitude_grad(circ, theta[p], kk))
        psi, dpsi = cache[(p, k)]
        x = W.x_index(vals[b, :circ.n])
        ref[b] = psi[x]
        assert abs(amp[b] - ref[b]) <= 1e-12, b
        assert np.max(np.abs(dft[b] - dpsi[:, x])) <= 1e-11, b
    _, p64 = g.eval(theta, ev, po, dtype="c64")
    ok, worst = prob_ok(p64.cpu().numpy(), np.abs(ref) ** 2)
    note(f"  complex64 probabilities: worst relative error {worst:.2e}")
    assert ok


def test_dpll_gradient_workload_rows_match_the_oracle():
    # the 16-qubit p=2 DEP+AD circuit (the gradient workload's), compiled by
    # search: sampled rows of its evidence in complex128 and complex64
    cfg = W.config(3, small=True)
    circ = cfg["circuit"]
    g = graph(compile_circuit_dpll(circ))
    note(f"dpll 16-qubit p=2: {g.info['n_internal']} nodes, {g.info['n_super']} super-nodes")
    ev, po, th = cfg["evidence"], cfg["param_of"], cfg["theta"]
    rows = np.random.default_rng(5).choice(len(ev), size=48, replace=False)
    amp128, _ = g.eval(th, ev, po, dtype="c128")
    _, p64 = g.eval(th, ev, po, dtype="c64")
    amp128 = amp128.cpu().numpy()
    p64 = p64.cpu().numpy()
    vals = W.unpack_evidence(circ, ev[rows])
    ref = np.array([sim.amplitude(circ, th[po[r]], W.x_index(v[:circ.n]), v[circ.n:]) for r, v in zip(rows, vals)])
    assert np.max(np.abs(amp128[rows] - ref)) <= 1e-12
    ok, worst = prob_ok(p64[rows], np.abs(ref) ** 2)
    note(f"  complex64 probabilities: worst relative error {worst:.2e}")
    assert ok
