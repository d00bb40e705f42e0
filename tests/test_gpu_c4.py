"""Sampling the noise-free 32-qubit QAOA p=1 circuit (no exact P(x) exists at
this size): per-qubit marginals 1/2 and the bit-flip symmetry of MaxCut QAOA,
and every edge's <Z_i Z_j> against the oracle's exact light-cone value, all
within binomial confidence bounds."""
import numpy as np
import pytest

import workloads as W
from oracle import sim
from tests.gpu_common import graph, note, require_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _gpu():
    require_gpu()


def _bits(samples, n):
    x = samples.reshape(-1).view(np.uint64)
    return ((x[:, None] >> np.arange(n, dtype=np.uint64)) & np.uint64(1)).astype(np.int8)


def test_c4_samples_marginals_symmetry_and_lightcone_zz():
    cfg = W.config(4, small=True)
    circ = cfg["circuit"]
    n = circ.n
    note("c4: compile and sample 2 x 16384 chains, 30 sweeps")
    g = graph(circ)
    theta = cfg["theta"][:2]
    C = 16384
    out = g.sample(theta, chains_per_param=C, samples_per_chain=1, burn_in=29, thin=1, seed=404, dtype="c64",
                   cost_edges=circ.edges, want_cost=True)
    samples = out["samples"].cpu().numpy()
    cost = out["cost"].cpu().numpy()
    z = 5.0
    for p in range(theta.shape[0]):
        bits = _bits(samples[p], n)
        # marginals: P(x_q = 1) = 1/2 (the law is invariant under flipping every bit)
        m = bits.mean(axis=0)
        assert np.all(np.abs(m - 0.5) <= z * 0.5 / np.sqrt(C) * 1.2), m
        # flip symmetry: Hamming weights w and n - w equally likely
        w = bits.sum(axis=1)
        hist = np.bincount(w, minlength=n + 1).astype(float)
        a, b = hist[: n // 2], hist[n:n // 2:-1]
        keep = (a + b) >= 10
        chi2 = float(np.sum((a[keep] - b[keep]) ** 2 / (a[keep] + b[keep])))
        from scipy.stats import chi2 as chi2d
        assert chi2d.sf(chi2, int(keep.sum())) > 1e-4
        # <Z_i Z_j> on every edge vs the light cone (Bonferroni over the edges)
        spins = 1 - 2 * bits.astype(np.int64)
        for (i, j) in circ.edges:
            est = float(np.mean(spins[:, i] * spins[:, j]))
            ref = sim.qaoa_p1_zz_lightcone(circ.edges, theta[p, 0], theta[p, 1], i, j)
            sd = np.sqrt(max(1.0 - ref * ref, 1e-3) / C)
            assert abs(est - ref) <= z * sd, (p, i, j, est, ref)
        # the reported cost is the number of cut edges of each sample
        want = sum(((bits[:, i] ^ bits[:, j]).astype(np.int64)) for i, j in circ.edges)
        assert np.array_equal(cost[p], want.astype(np.float64))
