"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module holds no arithmetic of the method itself: it only describes
circuits as plain op lists, draws random graphs, angles, noise strengths and
evidence assignments from fixed seeds, and packs/unpacks evidence words.
Both the oracle (``oracle/``) and the compiled GPU path consume what it makes;
neither side's arithmetic lives here.

Workload shapes follow the paper's evaluation: QAOA MaxCut on random
3-regular graphs (Sec. 4, "Evaluation for Ideal Circuit Simulation"), with a
symmetric depolarizing channel after each gate for the noisy runs (Sec. 4,
"Evaluation for Noisy Circuit Simulation", and Sec. 3.3.3), here extended by
amplitude damping for the deeper noisy case.

Op-list format (one tuple per op, in circuit order):

    ("H", q)                      Hadamard on qubit q
    ("CNOT", c, t)                CNOT, control c, target t
    ("RZ", q, j, s)               RZ(s * theta[j]) on q
    ("RX", q, j, s)               RX(s * theta[j]) on q
    ("DEP", q, m)                 symmetric depolarizing, total prob noise[m]
    ("AD", q, m)                  amplitude damping, gamma = noise[m]
    ("PD", q, m)                  phase damping, gamma = noise[m]

Evidence variables, in this order: output qubits q0..q(n-1) (domain 2), then
one variable per channel in circuit order (domain 4 for DEP: I, X, Y, Z;
domain 2 for AD and PD: Kraus index 0/1).  Each variable owns a field of
ceil(log2(dom)) bits, packed LSB-first into 64-bit words; a field that would
straddle a word boundary starts the next word instead.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Sequence, Tuple

import numpy as np

MASTER_SEED = 20210419
_SUB = {"graph": 1, "angles": 2, "noise": 3, "sampler": 4, "evidence": 5, "arrivals": 6}

CHANNEL_KINDS = ("DEP", "AD", "PD")
CHANNEL_DOM = {"DEP": 4, "AD": 2, "PD": 2}


def sub_seed(kind: str, config: int) -> int:
    """Seed for one input stream of one workload configuration."""
    return MASTER_SEED + _SUB[kind] * 1000 + int(config)


@dataclass
class Circuit:
    """A noisy variational circuit as a plain op list (see module doc)."""

    n: int
    ops: List[tuple]
    n_angles: int
    noise: List[float]
    edges: List[Tuple[int, int]] = field(default_factory=list)
    name: str = ""
    couplings: List[float] = field(default_factory=list)   # Ising J per edge (VQE circuits)
    fields: List[float] = field(default_factory=list)      # Ising h per qubit (VQE circuits)

    # ---- evidence-variable bookkeeping (format only, no arithmetic) ----
    def channels(self) -> List[tuple]:
        return [op for op in self.ops if op[0] in CHANNEL_KINDS]

    def var_domains(self) -> List[int]:
        return [2] * self.n + [CHANNEL_DOM[op[0]] for op in self.channels()]

    def var_layout(self) -> Tuple[List[int], List[int], int]:
        """(bit_offset[v], bit_width[v], W words) for every evidence variable."""
        offs, widths = [], []
        pos = 0
        for d in self.var_domains():
            w = max(1, int(math.ceil(math.log2(d))))
            if (pos % 64) + w > 64:
                pos = (pos // 64 + 1) * 64
            offs.append(pos)
            widths.append(w)
            pos += w
        n_words = max(1, (pos + 63) // 64)
        return offs, widths, n_words

    @property
    def n_vars(self) -> int:
        return self.n + len(self.channels())

    @property
    def n_words(self) -> int:
        return self.var_layout()[2]

    def n_gates(self) -> int:
        return sum(1 for op in self.ops if op[0] not in CHANNEL_KINDS)


# ---------------------------------------------------------------------------
# evidence packing
# ---------------------------------------------------------------------------

def pack_evidence(circ: Circuit, values: np.ndarray) -> np.ndarray:
    """values [B, n_vars] ints (x bits then Kraus indices) -> uint64 [B, W]."""
    values = np.asarray(values, dtype=np.int64)
    if values.ndim == 1:
        values = values[None, :]
    offs, widths, W = circ.var_layout()
    B = values.shape[0]
    words = np.zeros((B, W), dtype=np.uint64)
    for v, (o, w) in enumerate(zip(offs, widths)):
        wi, sh = divmod(o, 64)
        words[:, wi] |= (values[:, v].astype(np.uint64) & np.uint64((1 << w) - 1)) << np.uint64(sh)
    return words


def unpack_evidence(circ: Circuit, words: np.ndarray) -> np.ndarray:
    """uint64 [B, W] -> values [B, n_vars] int64."""
    words = np.asarray(words, dtype=np.uint64)
    if words.ndim == 1:
        words = words[None, :]
    offs, widths, _ = circ.var_layout()
    out = np.zeros((words.shape[0], len(offs)), dtype=np.int64)
    for v, (o, w) in enumerate(zip(offs, widths)):
        wi, sh = divmod(o, 64)
        out[:, v] = ((words[:, wi] >> np.uint64(sh)) & np.uint64((1 << w) - 1)).astype(np.int64)
    return out


def x_index(bits: Sequence[int]) -> int:
    """Basis-state index of an output assignment, LSB = qubit 0."""
    return int(sum(int(b) << q for q, b in enumerate(bits)))


def x_bits(index: int, n: int) -> np.ndarray:
    return np.array([(index >> q) & 1 for q in range(n)], dtype=np.int64)


# ---------------------------------------------------------------------------
# graphs
# ---------------------------------------------------------------------------

def random_regular_graph(n: int, d: int, seed: int) -> List[Tuple[int, int]]:
    """Uniform-ish random d-regular simple graph by the pairing model with
    rejection; edges returned as sorted (i<j) pairs in lexicographic order."""
    if (n * d) % 2 or d >= n:
        raise ValueError("no simple d-regular graph with these sizes")
    rng = np.random.default_rng(seed)
    for _ in range(10000):
        stubs = np.repeat(np.arange(n), d)
        rng.shuffle(stubs)
        pairs = stubs.reshape(-1, 2)
        ok = True
        seen = set()
        for a, b in pairs:
            a, b = int(a), int(b)
            if a == b:
                ok = False
                break
            e = (min(a, b), max(a, b))
            if e in seen:
                ok = False
                break
            seen.add(e)
        if ok:
            return sorted(seen)
    raise RuntimeError("pairing model did not produce a simple graph")


def ring_graph(n: int) -> List[Tuple[int, int]]:
    return sorted({(min(i, (i + 1) % n), max(i, (i + 1) % n)) for i in range(n)})


def maxcut_cost(edges: Sequence[Tuple[int, int]], bits: np.ndarray) -> np.ndarray:
    """Number of cut edges for each row of an output-bit array [B, n]."""
    bits = np.asarray(bits)
    if bits.ndim == 1:
        bits = bits[None, :]
    c = np.zeros(bits.shape[0], dtype=np.int64)
    for i, j in edges:
        c += (bits[:, i] != bits[:, j]).astype(np.int64)
    return c


# ---------------------------------------------------------------------------
# circuits
# ---------------------------------------------------------------------------

def qaoa_maxcut(n: int, edges: Sequence[Tuple[int, int]], p: int,
                dep=None, ad=None, name: str = "") -> Circuit:
    """QAOA MaxCut circuit: H on every qubit, then per layer l: for each edge
    (i<j) in lexicographic order CNOT(i->j) RZ(2 gamma_l) on j CNOT(i->j), then
    RX(2 beta_l) on every qubit.  theta[2l] = gamma_l, theta[2l+1] = beta_l.

    dep: None, a float (one shared depolarizing strength) or a sequence with
    one strength per depolarizing channel.  ad: None or a float (shared).
    After every gate, each qubit the gate touches gets a depolarizing channel
    and then (if ad) an amplitude-damping channel.
    """
    edges = sorted((min(a, b), max(a, b)) for a, b in edges)
    ops: List[tuple] = []
    noise: List[float] = []
    per_channel_dep = dep is not None and not np.isscalar(dep)
    dep_list = list(dep) if per_channel_dep else None
    dep_count = [0]
    if dep is not None and not per_channel_dep:
        noise.append(float(dep))
    ad_idx = None
    if ad is not None:
        ad_idx = len(noise)
        noise.append(float(ad))

    def after(qs):
        for q in qs:
            if dep is not None:
                if per_channel_dep:
                    m = len(noise)
                    noise.append(float(dep_list[dep_count[0]]))
                    dep_count[0] += 1
                else:
                    m = 0
                ops.append(("DEP", q, m))
            if ad is not None:
                ops.append(("AD", q, ad_idx))

    for q in range(n):
        ops.append(("H", q))
        after([q])
    for l in range(p):
        for i, j in edges:
            ops.append(("CNOT", i, j))
            after([i, j])
            ops.append(("RZ", j, 2 * l, 2.0))
            after([j])
            ops.append(("CNOT", i, j))
            after([i, j])
        for q in range(n):
            ops.append(("RX", q, 2 * l + 1, 2.0))
            after([q])
    if per_channel_dep and dep_count[0] != len(dep_list):
        raise ValueError("need exactly one depolarizing strength per channel: "
                         f"got {len(dep_list)}, circuit has {dep_count[0]}")
    return Circuit(n=n, ops=ops, n_angles=2 * p, noise=noise, edges=list(edges), name=name)


def grid_graph(rows: int, cols: int) -> List[Tuple[int, int]]:
    """Nearest-neighbour edges of a rows x cols grid, qubit q = r * cols + c."""
    edges = []
    for r in range(rows):
        for c in range(cols):
            q = r * cols + c
            if c + 1 < cols:
                edges.append((q, q + 1))
            if r + 1 < rows:
                edges.append((q, q + cols))
    return sorted(edges)


def ising_instance(rows: int, cols: int, seed: int):
    """Random 2D Ising instance: grid edges with couplings J = +-1 and a
    field h = +-1 on every site, uniform from the seed."""
    rng = np.random.default_rng(seed)
    edges = grid_graph(rows, cols)
    J = [float(v) for v in rng.choice([-1.0, 1.0], size=len(edges))]
    h = [float(v) for v in rng.choice([-1.0, 1.0], size=rows * cols)]
    return edges, J, h


def ising_energy(edges, J, h, bits: np.ndarray) -> np.ndarray:
    """E(x) = sum_(i,j) J_ij s_i s_j + sum_i h_i s_i with s = 1 - 2x, for bits [B, n]."""
    spins = 1 - 2 * np.asarray(bits, dtype=np.int64)
    e = np.zeros(spins.shape[0])
    for (i, j), Jij in zip(edges, J):
        e += Jij * spins[:, i] * spins[:, j]
    for i, hi in enumerate(h):
        e += hi * spins[:, i]
    return e


def vqe_ising(rows: int, cols: int, p: int, J: Sequence[float], h: Sequence[float],
              dep=None, ad=None, name: str = "") -> Circuit:
    """Variational circuit for the 2D Ising model: one qubit per grid site,
    two-qubit gates on the grid couplings.  H on every qubit, then per
    iteration l: for each edge (i<j) CNOT(i->j) RZ(2 J_ij gamma_l) on j
    CNOT(i->j) (the coupling phase exp(-i gamma_l J_ij Z_i Z_j)), RZ(2 h_i
    beta_l) on every qubit (the field), RX(2 alpha_l) on every qubit.
    theta[3l] = gamma_l, theta[3l+1] = beta_l, theta[3l+2] = alpha_l.
    Noise as in ``qaoa_maxcut`` (dep / ad after every gate on the qubits it
    touches; one shared strength each)."""
    n = rows * cols
    edges = grid_graph(rows, cols)
    if len(J) != len(edges) or len(h) != n:
        raise ValueError("need one coupling per grid edge and one field per site")
    ops: List[tuple] = []
    noise: List[float] = []
    if dep is not None:
        noise.append(float(dep))
    ad_idx = None
    if ad is not None:
        ad_idx = len(noise)
        noise.append(float(ad))

    def after(qs):
        for q in qs:
            if dep is not None:
                ops.append(("DEP", q, 0))
            if ad is not None:
                ops.append(("AD", q, ad_idx))

    for q in range(n):
        ops.append(("H", q))
        after([q])
    for l in range(p):
        for (i, j), Jij in zip(edges, J):
            ops.append(("CNOT", i, j))
            after([i, j])
            ops.append(("RZ", j, 3 * l, 2.0 * float(Jij)))
            after([j])
            ops.append(("CNOT", i, j))
            after([i, j])
        for q in range(n):
            ops.append(("RZ", q, 3 * l + 1, 2.0 * float(h[q])))
            after([q])
        for q in range(n):
            ops.append(("RX", q, 3 * l + 2, 2.0))
            after([q])
    return Circuit(n=n, ops=ops, n_angles=3 * p, noise=noise, edges=list(edges),
                   name=name or f"vqe_ising_{rows}x{cols}_p{p}", couplings=[float(v) for v in J],
                   fields=[float(v) for v in h])


def qaoa_channel_count(n: int, n_edges: int, p: int) -> int:
    """Number of single-qubit channel slots (one per touched qubit per gate)."""
    return n + p * (5 * n_edges + n)


def random_circuit(seed: int, n: int = None, n_ops: int = None, n_angles: int = 3, n_noise: int = 3) -> Circuit:
    """A seeded random op list over every op kind: H, CNOT in either
    direction, RZ/RX with random angle indices and scales (negative and
    non-unit included), and DEP/AD/PD channels at random places with
    strengths ~ U[0.02, 0.3]."""
    rng = np.random.default_rng(seed)
    n = int(rng.integers(2, 6)) if n is None else n
    n_ops = int(rng.integers(12, 31)) if n_ops is None else n_ops
    kinds = ["H", "CNOT", "RZ", "RX", "DEP", "AD", "PD"]
    weights = np.array([2, 3, 3, 3, 1, 1, 1], dtype=float)
    ops = [("H", q) for q in range(n) if rng.uniform() < 0.5]
    for _ in range(n_ops):
        k = kinds[int(rng.choice(len(kinds), p=weights / weights.sum()))]
        q = int(rng.integers(0, n))
        if k == "H":
            ops.append(("H", q))
        elif k == "CNOT":
            t = int(rng.integers(0, n - 1))
            ops.append(("CNOT", q, t if t < q else t + 1))
        elif k in ("RZ", "RX"):
            ops.append((k, q, int(rng.integers(0, n_angles)), float(rng.choice([-2.0, -1.0, 0.5, 1.0, 2.0, 3.0]))))
        else:
            ops.append((k, q, int(rng.integers(0, n_noise))))
    noise = [float(x) for x in rng.uniform(0.02, 0.3, size=n_noise)]
    return Circuit(n=n, ops=ops, n_angles=n_angles, noise=noise, name=f"random_{seed}")


def qaoa_ring_mpe(n: int = 4, dep: float = 0.02, ad: float = 0.05) -> Circuit:
    """Noise-free QAOA p=1 on the n-ring with amplitude damping after each H
    and depolarizing noise after each mixer RX (2n channels): a circuit for
    most-probable-explanation queries, small enough for the events-first
    compilation they need (n=4: 8 channels)."""
    base = qaoa_maxcut(n, ring_graph(n), 1)
    ops: List[tuple] = []
    for op in base.ops:
        ops.append(op)
        if op[0] == "H":
            ops.append(("AD", op[1], 1))
        elif op[0] == "RX":
            ops.append(("DEP", op[1], 0))
    return Circuit(n=n, ops=ops, n_angles=base.n_angles, noise=[dep, ad], edges=list(base.edges),
                   name=f"qaoa_ring{n}_mpe")


def noisy_bell(gamma: float = 0.36) -> Circuit:
    """The paper's running example (Sec. 3.1): H on q0, phase damping on q0,
    CNOT q0 -> q1."""
    return Circuit(n=2, ops=[("H", 0), ("PD", 0, 0), ("CNOT", 0, 1)], n_angles=0,
                   noise=[float(gamma)], edges=[], name="noisy_bell")


# ---------------------------------------------------------------------------
# configurations (shapes of the paper's QAOA workloads)
# ---------------------------------------------------------------------------

def uniform_angles(P: int, K: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return rng.uniform(0.0, 2.0 * np.pi, size=(P, K))


def sample_channel_prior(circ: Circuit, B: int, rng) -> np.ndarray:
    """Kraus indices [B, C] drawn from each channel's prior: DEP picks I with
    prob 1-p and X/Y/Z with p/3 each; AD/PD pick index 1 with prob gamma."""
    chans = circ.channels()
    k = np.zeros((B, len(chans)), dtype=np.int64)
    for c, op in enumerate(chans):
        pr = circ.noise[op[2]]
        u = rng.random(B)
        if op[0] == "DEP":
            k[:, c] = np.where(u < pr, 1 + rng.integers(0, 3, size=B), 0)
        else:
            k[:, c] = (u < pr).astype(np.int64)
    return k


def config(i: int, small: bool = False) -> dict:
    """Workload configuration i (1..5) as a dict of circuit + inputs.

    1: noise-free QAOA p=1 on the 4-ring; 64 angle pairs x all 16 outputs.
    2: QAOA p=1, random 3-regular n=8, depolarizing 0.01 after every gate;
       1024 angle pairs x 1000 samples each.
    3: QAOA p=2, random 3-regular n=16, depolarizing p_c ~ U[1e-3,1e-2] per
       channel + amplitude damping 5e-3; 4096 angle sets x 64 seeded (x,k).
    4: noise-free QAOA p=1, random 3-regular n=32; 256 angle pairs, ~1e6 samples.
    5: serving mix (see ``serving_pool``).
    small=True shrinks the batch dimensions (not the circuit) for quick tests.
    """
    if i == 1:
        edges = ring_graph(4)
        circ = qaoa_maxcut(4, edges, 1, name="qaoa_ring4_p1")
        P = 8 if small else 64
        theta = uniform_angles(P, 2, sub_seed("angles", 1))
        xs = np.arange(16)
        vals = np.stack([x_bits(x, 4) for x in xs])
        ev = pack_evidence(circ, vals)
        param_of = np.repeat(np.arange(P, dtype=np.int32), 16)
        evidence = np.tile(ev, (P, 1))
        return dict(circuit=circ, theta=theta, param_of=param_of, evidence=evidence,
                    dtype="c128", chains_per_param=None)
    if i == 2:
        edges = random_regular_graph(8, 3, sub_seed("graph", 2))
        circ = qaoa_maxcut(8, edges, 1, dep=0.01, name="qaoa_n8_p1_dep")
        P = 16 if small else 1024
        theta = uniform_angles(P, 2, sub_seed("angles", 2))
        return dict(circuit=circ, theta=theta, dtype="c64",
                    chains_per_param=(50 if small else 1000), samples_per_chain=1)
    if i == 3:
        n, p = 16, 2
        edges = random_regular_graph(n, 3, sub_seed("graph", 3))
        n_dep = qaoa_channel_count(n, len(edges), p)
        rng = np.random.default_rng(sub_seed("noise", 3))
        dep = rng.uniform(1e-3, 1e-2, size=n_dep)
        circ = qaoa_maxcut(n, edges, p, dep=dep, ad=5e-3, name="qaoa_n16_p2_dep_ad")
        P = 8 if small else 4096
        M = 64
        theta = uniform_angles(P, 4, sub_seed("angles", 3))
        erng = np.random.default_rng(sub_seed("evidence", 3))
        B = P * M
        xb = erng.integers(0, 2, size=(B, n))
        kk = sample_channel_prior(circ, B, erng)
        evidence = pack_evidence(circ, np.concatenate([xb, kk], axis=1))
        param_of = np.repeat(np.arange(P, dtype=np.int32), M)
        return dict(circuit=circ, theta=theta, param_of=param_of, evidence=evidence,
                    dtype="c64", chains_per_param=None)
    if i == 4:
        edges = random_regular_graph(32, 3, sub_seed("graph", 4))
        circ = qaoa_maxcut(32, edges, 1, name="qaoa_n32_p1")
        P = 4 if small else 256
        theta = uniform_angles(P, 2, sub_seed("angles", 4))
        return dict(circuit=circ, theta=theta, dtype="c64",
                    chains_per_param=(64 if small else 3907), samples_per_chain=1)
    raise ValueError(f"unknown config {i}")


def serving_pool(seed: int = None) -> List[Circuit]:
    """Pool of noisy QAOA circuits for the serving mix: p in {1,2},
    n in {6,8,12,16,20}, 4 seeded graphs each, one depolarizing strength
    ~U[1e-3,1e-2] per circuit."""
    seed = sub_seed("graph", 5) if seed is None else seed
    rng = np.random.default_rng(seed)
    pool = []
    for p in (1, 2):
        for n in (6, 8, 12, 16, 20):
            for g in range(4):
                edges = random_regular_graph(n, 3, int(rng.integers(1 << 31)))
                pr = float(rng.uniform(1e-3, 1e-2))
                pool.append(qaoa_maxcut(n, edges, p, dep=pr, name=f"qaoa_n{n}_p{p}_g{g}"))
    return pool


def log_uniform_int(rng, hi: int, size=None):
    """Integers in [1, hi] with log-uniform density: floor(exp(U[0, ln(hi+1))))."""
    v = np.floor(np.exp(rng.uniform(0.0, np.log(hi + 1.0), size=size))).astype(np.int64)
    return np.clip(v, 1, hi)


def serving_requests(pool: Sequence[Circuit], rate: float, duration: float, seed: int = None,
                     max_params: int = 256, max_samples: int = 4096, eval_rows: int = 64,
                     p_eval: float = 0.1, p_grad: float = 0.5) -> List[dict]:
    """Seeded request stream of the serving mix.

    Poisson arrivals at ``rate`` per second over ``duration`` seconds.  Each
    request: a circuit uniform from the pool; P ~ log-uniform{1..max_params}
    parameter sets ~ U[0, 2pi); with probability ``p_eval`` an amplitude
    request over ``eval_rows`` uniform outputs x with every noise event at
    its first value (k = 0) per parameter set, else S ~
    log-uniform{1..max_samples} samples per parameter set; a gradient with
    probability ``p_grad`` (for amplitude requests: of sum_b C(x_b) |f_b|^2;
    a sampled gradient needs two samples per set for its leave-one-out
    baseline, so its S is drawn from {2..max_samples}).
    """
    seed = sub_seed("arrivals", 5) if seed is None else seed
    rng = np.random.default_rng(seed)
    out = []
    t = 0.0
    while True:
        t += float(rng.exponential(1.0 / rate))
        if t >= duration:
            break
        ci = int(rng.integers(len(pool)))
        circ = pool[ci]
        P = int(log_uniform_int(rng, max_params))
        theta = rng.uniform(0.0, 2.0 * np.pi, size=(P, circ.n_angles))
        grad = bool(rng.random() < p_grad)
        r = dict(t=t, circuit=ci, theta=theta, grad=grad, samples=0, seed=int(rng.integers(1, 1 << 62)))
        if rng.random() < p_eval:
            B = P * eval_rows
            vals = np.zeros((B, circ.n_vars), dtype=np.int64)
            vals[:, :circ.n] = rng.integers(0, 2, size=(B, circ.n))
            r["evidence"] = pack_evidence(circ, vals)
            r["param_of"] = np.repeat(np.arange(P, dtype=np.int32), eval_rows)
            r["weight"] = maxcut_cost(circ.edges, vals[:, :circ.n]).astype(np.float64)
        else:
            r["samples"] = int(log_uniform_int(rng, max_samples))
            if grad and r["samples"] < 2:
                r["samples"] = 1 + int(log_uniform_int(rng, max_samples - 1))
        out.append(r)
    return out
