"""The paper's largest QAOA setting: noise-free p=2 MaxCut on a random
3-regular graph with 32 qubits.  Our compiler builds its AC with ~157k
internal nodes (the paper's compiler: 3.9M); Gibbs samples on the GPU are
checked against the exact p=2 reverse light cone (<Z_i Z_j> of every edge,
state vectors of at most 14 qubits), bit-flip symmetry and the MaxCut cost of
every sample."""
import numpy as np
import pytest

import workloads as W
from oracle import sim
from paper_2103_17226_amd.compiler import compile_circuit
from tests.gpu_common import graph, note, require_gpu

pytestmark = pytest.mark.gpu

N = 32


@pytest.fixture(autouse=True)
def _gpu():
    require_gpu()


def _bits(x):
    x = np.asarray(x).reshape(-1).view(np.uint64)
    return ((x[:, None] >> np.arange(N, dtype=np.uint64)) & np.uint64(1)).astype(np.int64)


def test_32_qubit_p2_samples_against_the_light_cone():
    edges = W.random_regular_graph(N, 3, W.sub_seed("graph", 4))
    circ = W.qaoa_maxcut(N, edges, 2)
    ac = compile_circuit(circ, order_trials=8)
    note(f"32-qubit p=2 QAOA: AC with {ac.n_internal} internal nodes, {ac.n_edges} edges, {ac.n_levels} levels")
    g = graph(ac)
    theta = np.array([[0.30, 0.25, 0.50, 0.20], [1.20, 0.90, 0.40, 0.60]])
    C = 4096
    out = g.sample(theta, C, 1, 20, 1, 3232, cost_edges=circ.edges, dtype="c64", want_cost=True)
    x = out["samples"].cpu().numpy().reshape(2, C)
    cost = out["cost"].cpu().numpy().reshape(2, C)
    g.release_workspaces()
    for p in range(2):
        bits = _bits(x[p])
        assert np.array_equal(cost[p], W.maxcut_cost(circ.edges, bits).astype(np.float64))
        spins = 1 - 2 * bits
        z = spins.mean(axis=0)
        assert np.all(np.abs(z) <= 5.0 / np.sqrt(C)), np.max(np.abs(z))
        worst = 0.0
        for (i, j) in circ.edges:
            est = float(np.mean(spins[:, i] * spins[:, j]))
            ref = sim.qaoa_zz_lightcone(circ.edges, theta[p], i, j)
            sd = np.sqrt(max(1.0 - ref * ref, 1e-3) / C)
            worst = max(worst, abs(est - ref) / sd)
            assert abs(est - ref) <= 5.0 * sd, (p, i, j, est, ref)
        note(f"  parameter set {p}: mean cost {cost[p].mean():.2f}, worst |<ZZ> - light cone| = {worst:.2f} sigma")
