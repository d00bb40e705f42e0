"""Search-based knowledge compilation of a circuit's factor graph into a
decision-DNNF, read as an arithmetic circuit (Sec. 3.2.2).

The paper compiles the circuit's CNF with c2d: an exhaustive DPLL search
that decides one variable at a time, splits the remaining constraints into
independent components, caches every component it has compiled, and orders
its decisions by a decomposition tree (dtree) of the constraints' hypergraph
obtained by recursive bisection.  This module runs that procedure on the
factor graph built by ``compiler.build_factors`` -- each factor is the set of
CNF clauses of one conditional amplitude table, its absent entries being the
excluded (zero) combinations -- and emits the same flat AC as the
variable-elimination compiler:

  * a decision on variable X is a sum node over its values x, each branch a
    product of the evidence indicator lambda_{X=x} (for evidence variables),
    the entries of the factors that X=x completes, and the compiled
    components of what remains; every variable of a component is decided on
    every path through it, so the result is smooth, and branches are
    disjoint (deterministic);
  * a component is a set of factors connected through undecided variables;
    components share no variable, so their product is decomposable;
  * a component is cached under its factors and the values of the decided
    variables its factors mention (its context), so equal sub-problems are
    compiled once and the result is a DAG;
  * the dtree splits the factors recursively into two halves that share few
    variables (a breadth-first seed order refined by single moves, the
    Fiduccia-Mattheyses idea), and a component decides first the undecided
    variables that its lowest covering dtree node cuts.
"""
from __future__ import annotations

import sys
import threading
from collections import defaultdict, deque
from typing import Dict, List, Optional, Tuple

from .compiler import CompiledAC, _elimination_order, build_factors, finish_compiled


# ---------------------------------------------------------------------------
# dtree: recursive hypergraph bisection of the factors
# ---------------------------------------------------------------------------

class DNode:
    __slots__ = ("factors", "left", "right", "cut", "lo", "hi")

    def __init__(self, factors, left=None, right=None, cut=()):
        self.factors = factors
        self.left, self.right = left, right
        self.cut = cut                      # variables shared by the two halves
        self.lo = self.hi = 0               # its leaves' positions [lo, hi) in depth-first order


def _bisect(fids: List[int], scopes: List[Tuple[int, ...]], passes: int = 4) -> Tuple[List[int], List[int]]:
    """Two halves of the factors sharing few variables: a breadth-first order
    from a peripheral factor cut in the middle, then passes of single moves
    that lower the number of cut variables (sizes kept within 40-60%)."""
    n = len(fids)
    by_var: Dict[int, List[int]] = defaultdict(list)
    for f in fids:
        for v in scopes[f]:
            by_var[v].append(f)

    def bfs(start):
        seen = {start: 0}
        q = deque([start])
        order = []
        while q:
            f = q.popleft()
            order.append(f)
            for v in scopes[f]:
                for g in by_var[v]:
                    if g not in seen:
                        seen[g] = seen[f] + 1
                        q.append(g)
        for f in fids:                          # disconnected factors last
            if f not in seen:
                seen[f] = 1 << 30
                order.append(f)
        return order
    far = bfs(fids[0])[-1]
    order = bfs(far)
    side = {f: (0 if i < n // 2 else 1) for i, f in enumerate(order)}
    cnt = {v: [0, 0] for v in by_var}
    for f in fids:
        for v in scopes[f]:
            cnt[v][side[f]] += 1
    size = [sum(1 for f in fids if side[f] == 0), 0]
    size[1] = n - size[0]
    lo, hi = int(0.4 * n), n - int(0.4 * n)
    for _ in range(passes):
        moved = False
        for f in order:
            s = side[f]
            if not lo <= size[s] - 1 <= hi or not lo <= size[1 - s] + 1 <= hi:
                continue
            gain = 0
            for v in scopes[f]:
                c = cnt[v]
                before = c[0] > 0 and c[1] > 0
                c2 = list(c)
                c2[s] -= 1
                c2[1 - s] += 1
                after = c2[0] > 0 and c2[1] > 0
                gain += int(before) - int(after)
            if gain > 0:
                side[f] = 1 - s
                size[s] -= 1
                size[1 - s] += 1
                for v in scopes[f]:
                    cnt[v][s] -= 1
                    cnt[v][1 - s] += 1
                moved = True
        if not moved:
            break
    left = [f for f in fids if side[f] == 0]
    right = [f for f in fids if side[f] == 1]
    if not left or not right:
        left, right = fids[:n // 2], fids[n // 2:]
    return left, right


def _join(a: DNode, b: DNode, scopes) -> DNode:
    va = set(v for f in a.factors for v in scopes[f])
    vb = set(v for f in b.factors for v in scopes[f])
    return DNode(a.factors | b.factors, a, b, tuple(sorted(va & vb)))


def dtree_bisect(scopes: List[Tuple[int, ...]]) -> Optional[DNode]:
    """The dtree over factors 0..len(scopes)-1 by recursive bisection."""
    def rec(fids):
        if len(fids) == 1:
            return DNode(frozenset(fids))
        a, b = _bisect(fids, scopes)
        return _join(rec(a), rec(b), scopes)
    return rec(list(range(len(scopes)))) if scopes else None


def dtree_from_order(scopes: List[Tuple[int, ...]], order: List[int]) -> Optional[DNode]:
    """The dtree of an elimination order: eliminating a variable joins every
    subtree that mentions it into one (smallest first), so a node's cut
    variables are at most the clique of the variable that created it."""
    trees = [DNode(frozenset([i])) for i in range(len(scopes))]
    tvars = [set(sc) for sc in scopes]
    alive = dict(enumerate(zip(trees, tvars)))
    nxt = len(trees)
    for x in order:
        ids = [i for i, (_, vs) in alive.items() if x in vs]
        if len(ids) < 2:
            continue
        ids.sort(key=lambda i: len(alive[i][0].factors))
        t, vs = alive.pop(ids[0])
        for i in ids[1:]:
            u, us = alive.pop(i)
            t = _join(t, u, scopes)
            vs = vs | us
        alive[nxt] = (t, vs)
        nxt += 1
    rest = sorted(alive.values(), key=lambda tv: len(tv[0].factors))
    if not rest:
        return None
    t = rest[0][0]
    for u, _ in rest[1:]:
        t = _join(t, u, scopes)
    return t


# ---------------------------------------------------------------------------
# exhaustive DPLL with components and caching
# ---------------------------------------------------------------------------

class _Search:
    def __init__(self, F, dtree: str, first=frozenset()):
        self.F = F
        self.first = first                  # variables decided before any other in a component
        self.ac = F.ac
        self.factors = F.live
        self.scopes = [f.vars for f in self.factors]
        self.by_var: Dict[int, List[int]] = defaultdict(list)
        for i, sc in enumerate(self.scopes):
            for v in sc:
                self.by_var[v].append(i)
        if dtree == "bisect":
            self.root = dtree_bisect(self.scopes)
        elif dtree == "order":
            self.root = dtree_from_order(self.scopes, _elimination_order(self.factors, F.dom))
        else:
            raise ValueError(f"unknown dtree method {dtree!r}")
        self.cache: Dict[tuple, object] = {}
        self.decisions = 0
        self.hits = 0
        # number the dtree's leaves depth-first: a node covers a contiguous
        # range, so "component inside node" is a test of the component's
        # smallest and largest leaf position
        self.pos = [0] * len(self.scopes)
        stack = [(self.root, False)] if self.root is not None else []
        k = 0
        while stack:
            t, done = stack.pop()
            if t.left is None:
                t.lo = k
                for f in t.factors:
                    self.pos[f] = k
                k += 1
                t.hi = k
                continue
            if done:
                t.lo, t.hi = t.left.lo, t.right.hi
                continue
            stack += [(t, True), (t.right, False), (t.left, False)]

    def entry(self, fid: int, asg: Dict[int, int]):
        f = self.factors[fid]
        return f.table.get(tuple(asg[v] for v in f.vars))        # None: a zero entry

    def components(self, fids, asg):
        """Connected components of the factors through undecided variables."""
        left = set(fids)
        out = []
        while left:
            start = left.pop()
            comp = [start]
            q = [start]
            while q:
                f = q.pop()
                for v in self.scopes[f]:
                    if v in asg:
                        continue
                    for g in self.by_var[v]:
                        if g in left:
                            left.discard(g)
                            comp.append(g)
                            q.append(g)
            out.append(frozenset(comp))
        return out

    def covering(self, comp, start):
        """The lowest dtree node that covers the component, searched from
        ``start`` (a node that covers it: the parent component's)."""
        lo = min(self.pos[f] for f in comp)
        hi = max(self.pos[f] for f in comp) + 1
        t = start
        while t.left is not None:
            if t.left.lo <= lo and hi <= t.left.hi:
                t = t.left
            elif t.right.lo <= lo and hi <= t.right.hi:
                t = t.right
            else:
                break
        return t

    def choose(self, comp, asg, t):
        """The next decision: an undecided variable cut by dtree node t (the
        lowest that covers the component; most occurrences in it first);
        with ``first`` variables left in the component, one of them."""
        if self.first:
            occ: Dict[int, int] = defaultdict(int)
            for f in comp:
                for v in self.scopes[f]:
                    if v not in asg and v in self.first:
                        occ[v] += 1
            if occ:
                return max(occ, key=lambda v: (occ[v], -v))
        if t is not None and t.left is not None:
            cand = [v for v in t.cut if v not in asg and any(f in comp for f in self.by_var[v])]
            if cand:
                return max(cand, key=lambda v: (sum(1 for f in self.by_var[v] if f in comp), -v))
        occ: Dict[int, int] = defaultdict(int)
        for f in comp:
            for v in self.scopes[f]:
                if v not in asg:
                    occ[v] += 1
        return max(occ, key=lambda v: (occ[v], -v))

    def compile(self, comp, asg, start=None):
        """AC node (or ONE) of a component under the decisions asg; None if
        zero.  ``start``: a dtree node covering the component."""
        ctx_vars = sorted({v for f in comp for v in self.scopes[f] if v in asg})
        key = (comp, tuple(asg[v] for v in ctx_vars))
        hit = self.cache.get(key, self)
        if hit is not self:
            self.hits += 1
            return hit
        t = self.covering(comp, start if start is not None else self.root) if self.root is not None else None
        x = self.choose(comp, asg, t)
        self.decisions += 1
        branches = []
        for val in range(self.F.dom[x]):
            asg[x] = val
            items = []
            ok = True
            if x in self.F.indicator_of:
                items.append(self.ac.indicator(self.F.indicator_of[x], val))
            # only factors that mention x can have become complete (the
            # component holds no complete factor); the others remain
            done = [f for f in self.by_var[x] if f in comp and all(v in asg for v in self.scopes[f])]
            for f in sorted(done):
                e = self.entry(f, asg)
                if e is None:
                    ok = False
                    break
                items.append(e)
            rest = comp.difference(done) if done else comp
            if ok:
                for c in self.components(rest, asg):
                    r = self.compile(c, asg, t)
                    if r is None:
                        ok = False
                        break
                    items.append(r)
            del asg[x]
            if ok:
                p = self.ac.product(items)
                if p is not None:
                    branches.append(p)
        res = self.ac.total(branches) if branches else None
        self.cache[key] = res
        return res


def _deep(fn, depth: int = 100000, stack_bytes: int = 512 << 20):
    """Run fn in a thread with a large stack and recursion limit (the search
    recurses once per decision and component along a path)."""
    out = {}

    def run():
        limit = sys.getrecursionlimit()
        sys.setrecursionlimit(max(limit, depth))
        try:
            fn()
        except BaseException as exc:       # re-raised in the caller
            out["exc"] = exc
        finally:
            sys.setrecursionlimit(limit)
    old = threading.stack_size(stack_bytes)
    try:
        t = threading.Thread(target=run, name="dpll")
        t.start()
    finally:
        threading.stack_size(old)
    t.join()
    if "exc" in out:
        raise out["exc"]


def compile_circuit_dpll(circ, flatten: bool = True, selectors: bool = True,
                         dtree: str = "order", mpe: bool = False) -> CompiledAC:
    """Compile a circuit (op-list form) with the search-based compiler; the
    same flat AC format and polynomial as ``compiler.compile_circuit``.
    dtree: "order" builds the decomposition tree from the min-fill/min-weight
    elimination order, "bisect" by recursive hypergraph bisection.

    mpe=True compiles for most-probable-explanation queries over the noise
    events (Sec. 5): every event is an explicit variable (no selector
    leaves) and a component decides its events before any other variable,
    so every sum with an event below it is a decision on one evidence
    variable and the sums over hidden qubit values sit below all event
    decisions.  Max-product over the events is then exact on the AC
    (|a b|^2 = |a|^2 |b|^2 over the disjoint events of a product's
    children; a decision's branches are disjoint).  The search then
    enumerates joint event values per component, so the size grows
    exponentially with the events that share hidden variables."""
    if mpe:
        selectors = False
    F = build_factors(circ, selectors)
    first = frozenset(v for v, e in F.indicator_of.items() if e >= circ.n) if mpe else frozenset()
    S = _Search(F, dtree, first)
    parts = list(F.const_parts)
    _deep(lambda: parts.extend(S.compile(c, {}) for c in S.components(range(len(S.factors)), {})))
    if any(p is None for p in parts):
        raise ValueError("the compiled circuit is identically zero")
    root = F.ac.product(parts)
    if root is None:
        raise ValueError("the compiled circuit is identically zero")
    return finish_compiled(circ, F.bn, F.ac, root, F.ev_nodes, flatten,
                           dict(fg_vars=F.n_fg_vars, compiler="dpll", dtree=dtree, mpe=mpe, decisions=S.decisions, cache_hits=S.hits,
                                cache_entries=len(S.cache)))
