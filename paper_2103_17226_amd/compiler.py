"""Circuit -> Bayesian network -> CNF -> arithmetic circuit (CPU preprocessing).

The AC is compiled once per circuit structure and queried many times with new
parameters and evidence (Sec. 3.2).  This module is plain host code; its
output is a level-ordered CSR DAG that the GPU library loads (``blob.py``).

Stages
------
1. Quantum Bayesian network (Sec. 3.1): one node per initial qubit state and
   one per gate (the new state of the qubit the gate writes); each noise
   channel adds a noise-event node whose value selects the Kraus operator and
   a node for the qubit state after it.  A conditional amplitude table (CAT)
   is the transpose of the gate matrix, A(out = j | in = i) = U[j][i], and a
   permutation of it for CNOT (Table cat_hadamard, Table cat_cnot); a channel
   node has A(out = j | in = i, event = k) = E_k[j][i].
2. CNF (Sec. 3.2.1, Table bn_to_cnf): indicator variables for every node
   value, one weight variable per non-deterministic table entry, with the
   three simplifications of that section: known initial values substituted,
   0/1 entries turned into logic, numeric parameters replaced by weight
   variables resolved at query time.  ``to_cnf`` emits DIMACS text; it is the
   fidelity artefact of that stage and is checked by weighted model counting.
3. AC (Sec. 3.2.2): a sum-product DAG over indicator leaves (output qubits
   and noise events) and weight leaves (slots).  It is built by symbolic
   variable elimination on the network's factors (the exact-inference route
   the authors started from, Sec. 3.2), with sparse tables (deterministic
   zeros never stored), hash-consing, folding of constants, elision of
   intermediate qubit states by summing them out without indicators
   (Sec. 3.2.2, "qubit state elision") and an elimination order (Sec. 3.2.2,
   "elimination order") chosen as the cheapest of several seeded greedy runs
   (min-weight, min-fill, min-degree, randomised tie-breaks).  Gates whose tables are diagonal
   (RZ, phase damping, the control side of CNOT) do not open a new variable,
   which is the deterministic-entry simplification applied to qubit states.

The result is a polynomial in the indicators that is multilinear and smooth:
every monomial holds exactly one indicator per evidence variable, so the
derivative with respect to lambda_{v=u} at evidence s equals the amplitude of
s with v set to u (Sec. 3.3.2, downward pass).
"""
from __future__ import annotations

import heapq
import math
import random
from collections import defaultdict
from dataclasses import dataclass, field
from typing import Dict, List, Optional, Tuple

import numpy as np

CHANNEL_KINDS = ("DEP", "AD", "PD")
CHANNEL_DOM = {"DEP": 4, "AD": 2, "PD": 2}

# ---------------------------------------------------------------------------
# weight slots: numeric parameters resolved at query time
# ---------------------------------------------------------------------------
# base kinds (value before the coefficient)
B_CONST = 0      # (re, im) stored in the slot
B_COS = 1        # cos(s * theta[j] / 2)
B_SIN = 2        # sin(s * theta[j] / 2)
B_EXPM = 3       # exp(-i s theta[j] / 2)
B_EXPP = 4       # exp(+i s theta[j] / 2)
B_SQRT_1MP = 5   # sqrt(1 - noise[m])
B_SQRT_P3 = 6    # sqrt(noise[m] / 3)
B_SQRT_P = 7     # sqrt(noise[m])
ANGLE_BASES = (B_COS, B_SIN, B_EXPM, B_EXPP)
NOISE_BASES = (B_SQRT_1MP, B_SQRT_P3, B_SQRT_P)
# coefficient codes: value = coef * base
COEF = {0: 1.0 + 0j, 1: -1.0 + 0j, 2: 1j, 3: -1j}
COEF_CODE = {1.0 + 0j: 0, -1.0 + 0j: 1, 1j: 2, -1j: 3}


@dataclass(frozen=True)
class Slot:
    base: int
    index: int = 0            # angle index j or noise index m
    scale: float = 0.0        # angle scale s
    coef: int = 0             # COEF code
    re: float = 0.0           # B_CONST only
    im: float = 0.0

    @property
    def is_angle(self) -> bool:
        return self.base in ANGLE_BASES

    def value(self, theta, noise) -> complex:
        """Host-side value (used by the compiler's own checks only)."""
        b = self.base
        if b == B_CONST:
            v = complex(self.re, self.im)
        elif b == B_COS:
            v = math.cos(0.5 * self.scale * theta[self.index])
        elif b == B_SIN:
            v = math.sin(0.5 * self.scale * theta[self.index])
        elif b == B_EXPM:
            a = 0.5 * self.scale * theta[self.index]
            v = complex(math.cos(a), -math.sin(a))
        elif b == B_EXPP:
            a = 0.5 * self.scale * theta[self.index]
            v = complex(math.cos(a), math.sin(a))
        elif b == B_SQRT_1MP:
            v = math.sqrt(1.0 - noise[self.index])
        elif b == B_SQRT_P3:
            v = math.sqrt(noise[self.index] / 3.0)
        elif b == B_SQRT_P:
            v = math.sqrt(noise[self.index])
        else:
            raise ValueError(b)
        return COEF[self.coef] * v


ONE = ("one",)   # symbolic entry 1 (deterministic entry folded into logic)
INV_SQRT2 = 1.0 / math.sqrt(2.0)


def _const(v: complex) -> Slot:
    return Slot(B_CONST, re=float(v.real), im=float(v.imag))


def gate_cat(op) -> Dict[Tuple[int, int], object]:
    """Symbolic CAT of a single-qubit gate: {(in i, out j): entry}, entry
    is ONE or a Slot; zero entries are absent."""
    name = op[0]
    if name == "H":
        h = _const(INV_SQRT2)
        return {(0, 0): h, (0, 1): h, (1, 0): h, (1, 1): _const(-INV_SQRT2)}
    if name == "RX":
        j, s = op[2], float(op[3])
        c = Slot(B_COS, j, s)
        sn = Slot(B_SIN, j, s, coef=3)                      # -i sin
        return {(0, 0): c, (1, 1): c, (0, 1): sn, (1, 0): sn}
    if name == "RZ":
        j, s = op[2], float(op[3])
        return {(0, 0): Slot(B_EXPM, j, s), (1, 1): Slot(B_EXPP, j, s)}
    raise ValueError(name)


def channel_cat(op) -> Dict[Tuple[int, int, int], object]:
    """{(in i, event k, out j): entry} with entry = E_k[j][i]."""
    name, m = op[0], op[2]
    if name == "DEP":
        a = Slot(B_SQRT_1MP, m)
        return {
            (0, 0, 0): a, (1, 0, 1): a,                                  # I
            (0, 1, 1): Slot(B_SQRT_P3, m), (1, 1, 0): Slot(B_SQRT_P3, m),  # X
            (0, 2, 1): Slot(B_SQRT_P3, m, coef=2),                       # Y[1][0] = +i
            (1, 2, 0): Slot(B_SQRT_P3, m, coef=3),                       # Y[0][1] = -i
            (0, 3, 0): Slot(B_SQRT_P3, m), (1, 3, 1): Slot(B_SQRT_P3, m, coef=1),  # Z
        }
    if name == "AD":
        return {(0, 0, 0): ONE, (1, 0, 1): Slot(B_SQRT_1MP, m), (1, 1, 0): Slot(B_SQRT_P, m)}
    if name == "PD":
        return {(0, 0, 0): ONE, (1, 0, 1): Slot(B_SQRT_1MP, m), (1, 1, 1): Slot(B_SQRT_P, m)}
    raise ValueError(name)


# ---------------------------------------------------------------------------
# Stage 1: Bayesian network
# ---------------------------------------------------------------------------

@dataclass
class BNNode:
    name: str
    kind: str                 # "init", "gate", "event", "channel"
    dom: int
    parents: List[int]
    cat: Dict[tuple, object]  # (parent values..., own value) -> entry (ONE/Slot); zeros absent
    qubit: int = -1


@dataclass
class BayesNet:
    nodes: List[BNNode]
    outputs: List[int]        # node id of the final state of each qubit
    events: List[int]         # node id of each noise event (circuit order)
    n: int


def circuit_to_bn(circ) -> BayesNet:
    nodes: List[BNNode] = []
    cur = []
    for q in range(circ.n):
        nodes.append(BNNode(f"q{q}m0", "init", 2, [], {(0,): ONE}, q))
        cur.append(len(nodes) - 1)
    moment = [1] * circ.n
    events = []
    for op in circ.ops:
        name = op[0]
        if name == "CNOT":
            c, t = op[1], op[2]
            cat = {(a, b, a ^ b): ONE for a in (0, 1) for b in (0, 1)}
            nodes.append(BNNode(f"q{t}m{moment[t]}", "gate", 2, [cur[c], cur[t]], cat, t))
            cur[t] = len(nodes) - 1
            moment[t] += 1
        elif name in CHANNEL_KINDS:
            q = op[1]
            d = CHANNEL_DOM[name]
            nodes.append(BNNode(f"q{q}m{moment[q]}rv", "event", d, [],
                                {(k,): ONE for k in range(d)}, q))
            ev = len(nodes) - 1
            events.append(ev)
            cat = {(i, k, j): e for (i, k, j), e in channel_cat(op).items()}
            nodes.append(BNNode(f"q{q}m{moment[q]}", "channel", 2, [cur[q], ev], cat, q))
            cur[q] = len(nodes) - 1
            moment[q] += 1
        else:
            q = op[1]
            cat = {(i, j): e for (i, j), e in gate_cat(op).items()}
            nodes.append(BNNode(f"q{q}m{moment[q]}", "gate", 2, [cur[q]], cat, q))
            cur[q] = len(nodes) - 1
            moment[q] += 1
    return BayesNet(nodes=nodes, outputs=list(cur), events=events, n=circ.n)


def bn_node_count(bn: BayesNet) -> int:
    """Nodes excluding noise-event nodes (initial states + one per gate/channel)."""
    return sum(1 for nd in bn.nodes if nd.kind != "event")


# ---------------------------------------------------------------------------
# Stage 2: CNF (DIMACS) with indicator and weight variables
# ---------------------------------------------------------------------------

@dataclass
class CNF:
    n_vars: int
    clauses: List[List[int]]
    indicator: Dict[Tuple[int, int], int]      # (bn node, value) -> cnf var
    weight_var: Dict[int, Slot]                # cnf var -> parameter it stands for

    def dimacs(self) -> str:
        lines = [f"p cnf {self.n_vars} {len(self.clauses)}"]
        for v, s in sorted(self.weight_var.items()):
            lines.append(f"c weight {v} {s}")
        lines += [" ".join(map(str, c)) + " 0" for c in self.clauses]
        return "\n".join(lines) + "\n"


def to_cnf(bn: BayesNet) -> CNF:
    """Table bn_to_cnf: each node takes exactly one value; known initial
    values become unit clauses; a table entry that is 0 forbids its row; an
    entry that is 1 needs no weight variable; any other entry gets a weight
    variable that is true exactly when its row holds."""
    ind = {}
    nv = 0
    for i, nd in enumerate(bn.nodes):
        for u in range(nd.dom):
            nv += 1
            ind[(i, u)] = nv
    clauses: List[List[int]] = []
    weights: Dict[int, Slot] = {}
    for i, nd in enumerate(bn.nodes):
        vals = [ind[(i, u)] for u in range(nd.dom)]
        clauses.append(list(vals))                                  # at least one
        for a in range(nd.dom):
            for b in range(a + 1, nd.dom):
                clauses.append([-vals[a], -vals[b]])                # at most one
        if nd.kind == "init":
            clauses.append([ind[(i, 0)]])                          # known initial value
            continue
        doms = [bn.nodes[p].dom for p in nd.parents] + [nd.dom]
        for row in np.ndindex(*doms):
            lits = [ind[(p, row[t])] for t, p in enumerate(nd.parents)] + [ind[(i, row[-1])]]
            e = nd.cat.get(tuple(row))
            if e is None:
                clauses.append([-l for l in lits])                 # zero entry: row impossible
            elif e is ONE:
                continue
            else:
                nv += 1
                weights[nv] = e
                clauses.append([-l for l in lits] + [nv])          # row -> weight
                for l in lits:
                    clauses.append([-nv, l])                       # weight -> row
    return CNF(nv, clauses, ind, weights)


# ---------------------------------------------------------------------------
# Stage 3: symbolic variable elimination -> AC
# ---------------------------------------------------------------------------

OP_SUM, OP_PROD = 0, 1
LEAF_IND, LEAF_SLOT, LEAF_SEL = 2, 3, 4
NO_SLOT = -1


class ACBuilder:
    """Hash-consed DAG store.  Node ids are ints; leaves and internal nodes
    share one id space."""

    def __init__(self):
        self.kind: List[int] = []
        self.data: List[tuple] = []
        self.memo: Dict[tuple, int] = {}
        self.slots: List[Slot] = []
        self.slot_ids: Dict[Slot, int] = {}

    def _get(self, kind, data):
        key = (kind, data)
        nid = self.memo.get(key)
        if nid is None:
            nid = len(self.kind)
            self.kind.append(kind)
            self.data.append(data)
            self.memo[key] = nid
        return nid

    def slot_id(self, s: Slot) -> int:
        sid = self.slot_ids.get(s)
        if sid is None:
            sid = len(self.slots)
            self.slots.append(s)
            self.slot_ids[s] = sid
        return sid

    def slot(self, s: Slot) -> int:
        return self._get(LEAF_SLOT, (self.slot_id(s),))

    def indicator(self, var: int, val: int) -> int:
        return self._get(LEAF_IND, (var, val))

    def selector(self, var: int, slots: Tuple[int, ...]) -> int:
        """Leaf sum_u lambda_{var=u} * W[slots[u]] (NO_SLOT: zero entry).
        For one-hot evidence it selects the weight of the variable's value."""
        return self._get(LEAF_SEL, (var, tuple(slots)))

    def const_value(self, nid) -> Optional[complex]:
        if self.kind[nid] == LEAF_SLOT:
            s = self.slots[self.data[nid][0]]
            if s.base == B_CONST:
                return complex(s.re, s.im)
        return None

    def product(self, items: List[object]) -> Optional[int]:
        """items: node ids or ONE; returns node id, ONE, or None for zero."""
        c = 1.0 + 0j
        kids = []
        for it in items:
            if it is ONE:
                continue
            cv = self.const_value(it)
            if cv is not None:
                c *= cv
                continue
            kids.append(it)
        if c == 0:
            return None
        if abs(c - 1.0) > 0:
            kids.append(self.slot(_const(c)))
        if not kids:
            return ONE
        if len(kids) == 1:
            return kids[0]
        return self._get(OP_PROD, tuple(sorted(kids)))

    def total(self, items: List[object]) -> Optional[int]:
        kids = []
        c = 0j
        for it in items:
            if it is None:
                continue
            if it is ONE:
                c += 1.0
                continue
            cv = self.const_value(it)
            if cv is not None:
                c += cv
                continue
            kids.append(it)
        if c != 0:
            kids.append(ONE if c == 1.0 else self.slot(_const(c)))
        kids = [k for k in kids if k is not None]
        if not kids:
            return None
        if len(kids) == 1:
            return kids[0]
        if any(k is ONE for k in kids):
            kids = [self.slot(_const(1.0)) if k is ONE else k for k in kids]
        return self._get(OP_SUM, tuple(sorted(kids)))


@dataclass
class Factor:
    vars: Tuple[int, ...]
    table: Dict[Tuple[int, ...], object]     # assignment -> node id / ONE


def _restrict(f: Factor, var: int, val: int) -> Factor:
    if var not in f.vars:
        return f
    p = f.vars.index(var)
    nv = f.vars[:p] + f.vars[p + 1:]
    tab = {}
    for a, e in f.table.items():
        if a[p] == val:
            tab[a[:p] + a[p + 1:]] = e
    return Factor(nv, tab)


def _join_sum(ac: ACBuilder, factors: List[Factor], x: int, dom: Dict[int, int],
              indicator_of: Dict[int, int]) -> Factor:
    """Multiply the factors that mention x, multiply in x's indicator if x is
    an evidence variable, and sum x out.  Sparse hash join."""
    # running join: list of (assignment dict, list of entries)
    scope: List[int] = []
    rows = [({}, [])]
    for f in sorted(factors, key=lambda f: len(f.table)):
        shared = [v for v in f.vars if v in scope]
        new = [v for v in f.vars if v not in scope]
        index = defaultdict(list)
        for a, e in f.table.items():
            key = tuple(a[f.vars.index(v)] for v in shared)
            index[key].append((a, e))
        out = []
        for asg, ents in rows:
            key = tuple(asg[v] for v in shared)
            for a, e in index.get(key, ()):
                nasg = dict(asg)
                for v in new:
                    nasg[v] = a[f.vars.index(v)]
                out.append((nasg, ents + [e]))
        rows = out
        scope += new
    rest = tuple(sorted(v for v in scope if v != x))
    groups: Dict[tuple, List[object]] = defaultdict(list)
    ev = indicator_of.get(x)
    for asg, ents in rows:
        if ev is not None:
            ents = ents + [ac.indicator(ev, asg[x])]
        p = ac.product(ents)
        if p is None:
            continue
        groups[tuple(asg[v] for v in rest)].append(p)
    tab = {}
    for key, items in groups.items():
        s = ac.total(items)
        if s is not None:
            tab[key] = s
    return Factor(rest, tab)


def _greedy_order(factors: List[Factor], dom: Dict[int, int], crit: str, rng) -> Tuple[List[int], int]:
    """One greedy elimination order and its cost, the summed size of the
    eliminated cliques (the dense bound on every intermediate table).

    crit picks the primary score: "wf" = clique weight then fill-in, "fw" =
    fill-in then weight, "deg" = degree then weight; rng (or None) breaks the
    remaining ties at random."""
    adj: Dict[int, set] = defaultdict(set)
    for f in factors:
        for v in f.vars:
            adj[v]
            for w in f.vars:
                if w != v:
                    adj[v].add(w)
    alive = set(adj)

    def weight(v):
        w = dom[v]
        for u in adj[v]:
            w *= dom[u]
        return w

    def score(v):
        nb = list(adj[v])
        fill = 0
        for i in range(len(nb)):
            ai = adj[nb[i]]
            for j in range(i + 1, len(nb)):
                if nb[j] not in ai:
                    fill += 1
        w = weight(v)
        tie = rng.random() if rng is not None else 0.0
        if crit == "wf":
            return (w, fill, tie, v)
        if crit == "fw":
            return (fill, w, tie, v)
        return (len(nb), w, tie, v)

    current = {v: score(v) for v in alive}
    heap = list(current.values())
    heapq.heapify(heap)
    order, cost = [], 0
    while heap:
        s = heapq.heappop(heap)
        v = s[-1]
        if v not in alive or current[v] != s:
            continue
        cost += weight(v)
        order.append(v)
        alive.discard(v)
        nb = list(adj[v])
        for u in nb:
            adj[u].discard(v)
            for w in nb:
                if w != u:
                    adj[u].add(w)
        del adj[v]
        touched = set(nb)
        for u in nb:
            touched |= adj[u]
        for u in touched:
            if u in alive:
                current[u] = score(u)
                heapq.heappush(heap, current[u])
    return order, cost


# Larger circuits get more order trials: past ORDER_BIG summed clique size
# (an AC of roughly that many nodes) the search goes on in rounds of `trials`
# runs while a round still lowers the cost by ORDER_GAIN, up to ORDER_MAX_TRIALS
# runs -- a trial costs milliseconds, a node of the AC tens of microseconds.
ORDER_BIG = 2e5
ORDER_GAIN = 0.02
ORDER_MAX_TRIALS = 2048


def _elimination_order(factors: List[Factor], dom: Dict[int, int], trials: int = 64,
                       seed: int = 0x5EED) -> List[int]:
    """Elimination order (Sec. 3.2.2): the cheapest of several greedy runs.

    The three deterministic heuristics run first, then randomised tie-breaks
    of each in turn; the order with the smallest summed clique size wins
    (earliest on ties).  The number of runs depends only on the costs found,
    so the result is reproducible."""
    rng = random.Random(seed)
    crits = ("wf", "fw", "deg")
    best = None
    t = 0
    n = max(1, trials)
    while True:
        round_start = None if best is None else best[1]
        for _ in range(n):
            order, cost = _greedy_order(factors, dom, crits[t % 3], rng if t >= 3 else None)
            if best is None or cost < best[1]:
                best = (order, cost)
            t += 1
        if best[1] <= ORDER_BIG or t >= ORDER_MAX_TRIALS or trials <= 1:
            break
        if round_start is not None and best[1] > (1.0 - ORDER_GAIN) * round_start:
            break
    return best[0]


@dataclass
class CompiledAC:
    """Flat AC: internal nodes in level order, tagged child refs, slot table,
    evidence-variable table."""
    n_qubits: int
    var_dom: List[int]
    var_kind: List[int]           # 0 output, 1 DEP event, 2 AD event, 3 PD event
    var_offset: List[int]
    n_words: int
    n_angles: int
    n_noise: int
    noise_default: List[float]
    slots: List[Slot]
    selectors: List[Tuple[int, Tuple[int, ...]]]   # (variable, slot per value or NO_SLOT)
    op: np.ndarray                # uint8 [N_int]
    row_ptr: np.ndarray           # int32 [N_int + 1]
    col: np.ndarray               # uint32 [E] tagged child refs
    level_ptr: np.ndarray         # int32 [L + 1]
    root: int                     # internal index of the root
    stats: dict = field(default_factory=dict)

    @property
    def n_internal(self):
        return int(len(self.op))

    @property
    def n_edges(self):
        return int(len(self.col))

    @property
    def n_levels(self):
        return int(len(self.level_ptr) - 1)


# child-ref tags (top two bits)
TAG_NODE = 0
TAG_IND = 1
TAG_SLOT = 2
TAG_SEL = 3
TAG_SHIFT = 30
IND_VAL_SHIFT = 24          # indicator ref: var in bits 0..23, value in bits 24..29


def ref_node(i):
    return (TAG_NODE << TAG_SHIFT) | i


def ref_ind(v, u):
    return (TAG_IND << TAG_SHIFT) | (u << IND_VAL_SHIFT) | v


def ref_slot(s):
    return (TAG_SLOT << TAG_SHIFT) | s


def ref_sel(q):
    return (TAG_SEL << TAG_SHIFT) | q


def _var_layout(doms):
    offs, pos = [], 0
    for d in doms:
        w = max(1, int(math.ceil(math.log2(d))))
        if (pos % 64) + w > 64:
            pos = (pos // 64 + 1) * 64
        offs.append(pos)
        pos += w
    return offs, max(1, (pos + 63) // 64)


@dataclass
class _Factors:
    """The factor graph of a circuit, ready for a compiler: the BN, the AC
    store holding its weight leaves, the factors over hidden and evidence
    variables, constant parts, domains and the evidence variable of each
    factor-graph variable."""
    bn: object
    ac: object
    live: list
    const_parts: list
    dom: dict
    indicator_of: dict
    ev_nodes: list
    n_fg_vars: int


def build_factors(circ, selectors: bool = True) -> _Factors:
    """Circuit -> BN (Sec. 3.1) -> factor graph with symbolic entries (the
    conditional amplitude tables, simplified as in Sec. 3.2.1): the common
    first stage of the variable-elimination and the search-based compilers."""
    bn = circuit_to_bn(circ)
    ac = ACBuilder()

    # --- evidence variables: outputs then events (circuit order)
    ev_nodes = list(bn.outputs) + list(bn.events)
    ev_index = {nd: i for i, nd in enumerate(ev_nodes)}

    # --- factor-graph variables: a BN node whose CAT is diagonal in its
    # qubit input shares the input's variable (no new variable).
    var_of: Dict[int, int] = {}
    dom: Dict[int, int] = {}
    factors: List[Factor] = []
    nvar = [0]

    def new_var(d):
        v = nvar[0]
        nvar[0] += 1
        dom[v] = d
        return v

    def sym(e):
        return ONE if e is ONE else ac.slot(e)

    known_zero: List[int] = []
    for i, nd in enumerate(bn.nodes):
        if nd.kind == "init":
            var_of[i] = new_var(2)
            known_zero.append(var_of[i])
            continue
        if nd.kind == "event":
            var_of[i] = new_var(nd.dom)
            continue
        parents = nd.parents
        # qubit input of this node: the last parent for gates (target for CNOT), first for channels
        if nd.kind == "channel":
            qin, extra = parents[0], [parents[1]]
        elif len(parents) == 2:
            qin, extra = parents[1], [parents[0]]
        else:
            qin, extra = parents[0], []
        if nd.kind == "channel":
            diagonal = all(key[0] == key[2] for key in nd.cat)       # (in, event, out)
        elif len(parents) == 1:
            diagonal = all(key[0] == key[1] for key in nd.cat)       # (in, out)
        else:
            diagonal = False                                         # CNOT target flips
        pv = [var_of[p] for p in parents]
        if nd.kind == "channel" and selectors:
            # Kraus selection: the event's indicators and the Kraus entries
            # E_k[j][i] fold into one selector leaf per (i, j) entry
            ev_var = ev_index[parents[1]]
            d = bn.nodes[parents[1]].dom
            per_entry: Dict[Tuple[int, int], List[int]] = {}
            for (a, k, b), e in nd.cat.items():
                lst = per_entry.setdefault((a, b), [NO_SLOT] * d)
                lst[k] = ac.slot_id(_const(1.0) if e is ONE else e)
            if diagonal:
                v = var_of[qin]
                tab = {(a,): ac.selector(ev_var, tuple(lst)) for (a, b), lst in per_entry.items()}
                fv = (v,)
            else:
                v = new_var(2)
                tab = {(a, b): ac.selector(ev_var, tuple(lst)) for (a, b), lst in per_entry.items()}
                fv = (pv[0], v)
            var_of[i] = v
            factors.append(Factor(fv, tab))
            continue
        if diagonal:
            v = var_of[qin]
            var_of[i] = v
            tab = {}
            for key, e in nd.cat.items():
                if nd.kind == "channel":
                    tab[(key[0], key[1])] = sym(e)       # (q, event)
                else:
                    tab[(key[0],)] = sym(e)
            fv = (v, pv[1]) if nd.kind == "channel" else (v,)
        else:
            v = new_var(2)
            var_of[i] = v
            tab = {key: sym(e) for key, e in nd.cat.items()}
            fv = tuple(pv) + (v,)
        factors.append(Factor(fv, tab))

    # known initial values (Sec. 3.2.1 simplification 1)
    for z in known_zero:
        factors = [_restrict(f, z, 0) for f in factors]
    zero_set = set(known_zero)

    indicator_of = {}
    for nd in ev_nodes:
        indicator_of[var_of[nd]] = ev_index[nd]
    # an output qubit left untouched by any gate is pinned to |0>: evidence
    # still needs its indicator -> unary factor lambda(v=0)
    for nd in bn.outputs:
        v = var_of[nd]
        if v in zero_set:
            e = ev_index[nd]
            factors.append(Factor((), {(): ac.indicator(e, 0)}))

    live = [f for f in factors if f.vars]
    const_parts = [f.table.get(()) for f in factors if not f.vars]
    return _Factors(bn, ac, live, const_parts, dom, indicator_of, ev_nodes, nvar[0])


def compile_circuit(circ, flatten: bool = True, selectors: bool = True,
                    order_trials: int = 64) -> CompiledAC:
    """Compile a circuit (op-list form) into a flat level-ordered AC.

    selectors=True folds each channel's event indicators and Kraus entries
    into selector leaves (one per matrix entry); False keeps them as sums of
    indicator x weight products.  Both give the same polynomial.
    order_trials is the number of greedy elimination-order runs to pick from
    (1 = plain min-weight/min-fill)."""
    F = build_factors(circ, selectors)
    bn, ac, live, const_parts, dom, indicator_of, ev_nodes = (F.bn, F.ac, F.live, list(F.const_parts), F.dom,
                                                               F.indicator_of, F.ev_nodes)
    # merge factors over identical scopes is implicit in VE
    order = _elimination_order(live, dom, order_trials)
    # variables that appear in no factor but are evidence: they must still carry an indicator
    bucket: Dict[int, List[Factor]] = defaultdict(list)
    pos = {v: i for i, v in enumerate(order)}
    for f in live:
        bucket[min(f.vars, key=lambda v: pos[v])].append(f)
    max_table = 0
    for x in order:
        fs = bucket.pop(x, [])
        if not fs:
            continue
        g = _join_sum(ac, fs, x, dom, indicator_of)
        max_table = max(max_table, len(g.table))
        if not g.vars:
            const_parts.append(g.table.get((), None))
            if g.table.get(()) is None:
                const_parts.append(None)
        else:
            bucket[min(g.vars, key=lambda v: pos[v])].append(g)
    if any(c is None for c in const_parts):
        root = None
    else:
        root = ac.product(const_parts)
    if root is None:
        raise ValueError("the compiled circuit is identically zero")

    return finish_compiled(circ, bn, ac, root, ev_nodes, flatten,
                           dict(fg_vars=F.n_fg_vars, max_table=max_table))


def finish_compiled(circ, bn, ac, root, ev_nodes, flatten: bool, stats: dict) -> "CompiledAC":
    """Level-ordered flat AC (the blob's form) from an AC store and its root."""
    var_dom = [bn.nodes[nd].dom for nd in ev_nodes]
    var_kind = [0] * bn.n + [{"DEP": 1, "AD": 2, "PD": 3}[op[0]] for op in circ.ops
                             if op[0] in CHANNEL_KINDS]
    offs, W = _var_layout(var_dom)
    out = _flatten_and_level(ac, root, flatten)
    op_arr, row_ptr, col, level_ptr, root_idx, slot_list, sel_list = out
    res = CompiledAC(n_qubits=bn.n, var_dom=var_dom, var_kind=var_kind, var_offset=offs,
                     n_words=W, n_angles=circ.n_angles, n_noise=len(circ.noise),
                     noise_default=list(circ.noise), slots=slot_list, selectors=sel_list,
                     op=op_arr, row_ptr=row_ptr, col=col, level_ptr=level_ptr, root=root_idx)
    res.stats = dict(bn_nodes=bn_node_count(bn), bn_events=len(bn.events), **stats,
                     n_internal=res.n_internal, n_edges=res.n_edges, n_levels=res.n_levels,
                     n_slots=len(slot_list), n_selectors=len(sel_list))
    return res


def _flatten_and_level(ac: ACBuilder, root, flatten: bool):
    """Reachable internal nodes from root; merge single-parent same-op
    children into their parent; assign levels; emit level-ordered CSR."""
    if root is ONE:
        root = ac.slot(_const(1.0))
    kind, data = ac.kind, ac.data
    # reachable + parent counts
    seen = set()
    stack = [root]
    order = []
    while stack:
        u = stack.pop()
        if u in seen:
            continue
        seen.add(u)
        order.append(u)
        if kind[u] in (OP_SUM, OP_PROD):
            stack.extend(data[u])
    nparents = defaultdict(int)
    for u in order:
        if kind[u] in (OP_SUM, OP_PROD):
            for c in data[u]:
                nparents[c] += 1
    children: Dict[int, List[int]] = {}

    def kids_of(u):
        if u in children:
            return children[u]
        out = []
        for c in data[u]:
            if flatten and kind[c] == kind[u] and nparents[c] == 1:
                out.extend(kids_of(c))
            else:
                out.append(c)
        children[u] = out
        return out

    # post-order over internal nodes after flattening
    internal = []
    state = {}
    if kind[root] not in (OP_SUM, OP_PROD):
        # degenerate AC: root is a leaf -> wrap in a 1-child product
        children[-1] = [root]
        kind_local = {-1: OP_PROD}
        internal = [-1]
        level = {-1: 1}
    else:
        kind_local = {}
        level = {}
        stack = [(root, False)]
        while stack:
            u, done = stack.pop()
            if done:
                lv = 0
                for c in kids_of(u):
                    if kind[c] in (OP_SUM, OP_PROD):
                        lv = max(lv, level[c])
                level[u] = lv + 1
                internal.append(u)
                continue
            if u in state:
                continue
            state[u] = 1
            stack.append((u, True))
            for c in kids_of(u):
                if kind[c] in (OP_SUM, OP_PROD) and c not in state:
                    stack.append((c, False))
    # order by level (stable in post-order within a level)
    internal.sort(key=lambda u: level[u])
    idx = {u: i for i, u in enumerate(internal)}
    # compact slot table: only slots referenced
    slot_map: Dict[int, int] = {}
    slot_list: List[Slot] = []
    sel_map: Dict[int, int] = {}
    sel_list: List[Tuple[int, Tuple[int, ...]]] = []

    def slot_ref_id(sid):
        if sid not in slot_map:
            slot_map[sid] = len(slot_list)
            slot_list.append(ac.slots[sid])
        return slot_map[sid]
    op_arr = np.zeros(len(internal), dtype=np.uint8)
    row_ptr = np.zeros(len(internal) + 1, dtype=np.int32)
    cols: List[int] = []
    for i, u in enumerate(internal):
        op_arr[i] = kind_local.get(u, kind[u] if u >= 0 else OP_PROD)
        refs = []
        for c in children[u] if u in children else kids_of(u):
            k = kind[c]
            if k in (OP_SUM, OP_PROD):
                refs.append(ref_node(idx[c]))
            elif k == LEAF_IND:
                v, val = data[c]
                refs.append(ref_ind(v, val))
            elif k == LEAF_SEL:
                if c not in sel_map:
                    v, sl = data[c]
                    sel_map[c] = len(sel_list)
                    sel_list.append((v, tuple(NO_SLOT if x == NO_SLOT else slot_ref_id(x) for x in sl)))
                refs.append(ref_sel(sel_map[c]))
            else:
                refs.append(ref_slot(slot_ref_id(data[c][0])))
        # internal children first (in index order), then leaves
        refs.sort(key=lambda r: (r >> TAG_SHIFT, r))
        cols.extend(refs)
        row_ptr[i + 1] = len(cols)
    lv = np.array([level[u] for u in internal], dtype=np.int64)
    L = int(lv.max()) if len(lv) else 0
    level_ptr = np.zeros(L + 1, dtype=np.int32)
    for l in range(1, L + 1):
        level_ptr[l] = int(np.searchsorted(lv, l, side="right"))
    return (op_arr, row_ptr, np.array(cols, dtype=np.uint32), level_ptr, idx[root] if root in idx else 0,
            slot_list, sel_list)
