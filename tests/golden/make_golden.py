"""Write the stored expected values under tests/golden/ from the oracle only.

    python tests/golden/make_golden.py

qaoa_n32_p1_pathsum.json: amplitudes of the 32-qubit noise-free QAOA p=1
workload (random 3-regular graph, seeded) at seeded (parameter set, x)
pairs, by the brute-force Feynman path sum over all 2^32 paths.
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import workloads as W  # noqa: E402
from oracle import pathsum  # noqa: E402


def qaoa_n32():
    cfg = W.config(4)
    circ = cfg["circuit"]
    theta = cfg["theta"]
    rng = np.random.default_rng(W.sub_seed("evidence", 4))
    xs = [int(v) for v in rng.integers(0, 1 << 32, size=8, dtype=np.uint64)]
    rows = []
    for x in xs:
        hist = pathsum.path_histogram(32, circ.edges, x)
        params = rng.choice(theta.shape[0], size=2, replace=False)
        amps = pathsum.amplitudes_from_histogram(hist, 32, len(circ.edges), theta[params, 0], theta[params, 1])
        for p, a in zip(params, amps):
            rows.append((int(p), x, complex(a)))
    used = sorted({p for p, _, _ in rows})
    remap = {p: i for i, p in enumerate(used)}
    out = {
        "_source": "Brute-force path sum (oracle/pathsum.c) over all 2^32 paths of noise-free QAOA p=1 "
                   "on the seeded 32-node random 3-regular graph; written by tests/golden/make_golden.py",
        "edges": [list(e) for e in circ.edges],
        "theta": [list(map(float, theta[p])) for p in used],
        "param": [remap[p] for p, _, _ in rows],
        "x": [str(x) for _, x, _ in rows],
        "amp_re": [a.real for _, _, a in rows],
        "amp_im": [a.imag for _, _, a in rows],
    }
    with open(os.path.join(HERE, "qaoa_n32_p1_pathsum.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    qaoa_n32()
