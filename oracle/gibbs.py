"""Gibbs sampling reference (Sec. 3.3.2) for the oracle.

Test infrastructure only (see ``oracle/__init__.py``).

The sampled state is an assignment s = (x, k) of the output qubits and the
noise-event variables, and its stationary weight is |f(x,k)|^2, so that the
x-marginal is P(x) = rho_xx.  Sec. 3.3.2 moves between assignments that
differ in one variable ("one away") with transition probabilities taken from
the downward pass, i.e. from the amplitudes of the neighbouring assignments.
The reading used here is single-site Gibbs with exact conditionals:

    P(v = u | rest) = |f(s[v <- u])|^2 / sum_u' |f(s[v <- u'])|^2

visited in a fixed systematic scan (outputs q0..q(n-1), then channels in
circuit order), one variable per decision.  A decision draws r in [0, 1) and
takes the smallest u with r * sum(w) < w_0 + ... + w_u; zero total mass keeps
the current value.

Randomness is the counter-based SplitMix64 finaliser (Steele, Lea and Flood,
"Fast splittable pseudorandom number generators", OOPSLA 2014), keyed by
(seed, chain, sweep, variable) so the device sampler can reproduce the same
stream from its own implementation:

    mix(z)   = finalise(z + 0x9E3779B97F4A7C15)
    finalise = z ^= z >> 30; z *= 0xBF58476D1CE4E5B9;
               z ^= z >> 27; z *= 0x94D049BB133111EB; z ^= z >> 31
    u(seed, chain, sweep, var) = (mix(seed ^ mix(chain ^ mix((sweep << 20) ^ var))) >> 11) * 2^-53

Chain initialisation: x_q = [u(seed, chain, INIT_SWEEP, q) < 1/2], k = 0.
Schedule: burn_in + S * thin sweeps; sample j is the state after sweep
burn_in + (j + 1) * thin.
"""
from __future__ import annotations

import numpy as np

from . import sim

MASK = (1 << 64) - 1
GOLDEN = 0x9E3779B97F4A7C15
INIT_SWEEP = 0xFFFFFFFF


def mix64(z: int) -> int:
    z = (z + GOLDEN) & MASK
    z ^= z >> 30
    z = (z * 0xBF58476D1CE4E5B9) & MASK
    z ^= z >> 27
    z = (z * 0x94D049BB133111EB) & MASK
    z ^= z >> 31
    return z


def uniform(seed: int, chain: int, sweep: int, var: int) -> float:
    inner = mix64((((sweep << 20) & MASK) ^ var) & MASK)
    mid = mix64((chain ^ inner) & MASK)
    top = mix64((seed ^ mid) & MASK)
    return (top >> 11) * (1.0 / 9007199254740992.0)


def choose(weights, r):
    """Inverse CDF on FP64 cumulative weights, strict '<', smallest u wins.
    Returns None for zero total mass (caller keeps the current value)."""
    total = 0.0
    for w in weights:
        total += w
    if not total > 0.0:
        return None
    target = r * total
    acc = 0.0
    last_pos = None
    for u, w in enumerate(weights):
        acc += w
        if w > 0.0:
            last_pos = u
        if target < acc:
            return u
    return last_pos


class BranchCache:
    """f(x, k) lookups backed by cached Kraus-branch state vectors."""

    def __init__(self, circ, theta, noise=None):
        self.circ, self.theta, self.noise = circ, np.asarray(theta, float), noise
        self.cache = {}

    def vector(self, k):
        key = tuple(int(v) for v in k)
        vec = self.cache.get(key)
        if vec is None:
            vec = sim.branch_state(self.circ, self.theta, key, self.noise)
            if len(self.cache) > 4096:
                self.cache.clear()
            self.cache[key] = vec
        return vec

    def amp(self, state):
        n = self.circ.n
        x = sum(int(state[q]) << q for q in range(n))
        return self.vector(state[n:])[x]


def conditional_weights(bc: BranchCache, state, v):
    """w_u = |f(s[v <- u])|^2 for every value u of variable v (FP64,
    computed as re*re + im*im)."""
    dom = bc.circ.var_domains()[v]
    out = []
    s = list(state)
    for u in range(dom):
        s[v] = u
        a = bc.amp(s)
        out.append(a.real * a.real + a.imag * a.imag)
    return out


def init_state(circ, seed, chain):
    s = [0] * circ.n_vars
    for q in range(circ.n):
        s[q] = 1 if uniform(seed, chain, INIT_SWEEP, q) < 0.5 else 0
    return s


def run_chain(circ, theta, seed, chain, burn_in, thin, n_samples, noise=None, init=None, first_sweep=0,
              first_var=0):
    """Reference systematic-scan chain; returns (samples [S, n_vars], final state).

    ``init`` (one value per variable) replaces the seeded start and
    ``first_sweep`` numbers the first sweep of this run in the random stream,
    so a run resumed from another run's final state with its sweep count
    continues that chain.  Variables before ``first_var`` are never updated
    (the chain then targets the conditional law of the others given them)."""
    bc = BranchCache(circ, theta, noise)
    s = init_state(circ, seed, chain) if init is None else [int(v) for v in init]
    V = circ.n_vars
    samples = []
    total = burn_in + n_samples * thin
    for sweep in range(total):
        for v in range(first_var, V):
            w = conditional_weights(bc, s, v)
            u = choose(w, uniform(seed, chain, first_sweep + sweep, v))
            if u is not None:
                s[v] = u
        done = sweep + 1
        if done > burn_in and (done - burn_in) % thin == 0:
            samples.append(list(s))
    return np.array(samples, dtype=np.int64), s


# ---------------------------------------------------------------------------
# exact finite-step distribution on tiny state spaces
# ---------------------------------------------------------------------------

def enumerate_states(circ):
    doms = circ.var_domains()
    grids = np.meshgrid(*[np.arange(d) for d in doms], indexing="ij")
    return np.stack([g.reshape(-1) for g in grids], axis=1)


def exact_sweep_distribution(circ, theta, sweeps, noise=None):
    """Distribution over all states after `sweeps` systematic-scan sweeps,
    starting from x uniform, k = 0.  Returns (states [N, V], probs [N])."""
    states = enumerate_states(circ)
    doms = circ.var_domains()
    index = {tuple(s): i for i, s in enumerate(states.tolist())}
    bc = BranchCache(circ, theta, noise)
    N = len(states)
    weight = np.array([abs(bc.amp(s)) ** 2 for s in states.tolist()])
    dist = np.zeros(N)
    for i, s in enumerate(states.tolist()):
        if all(val == 0 for val in s[circ.n:]):
            dist[i] = 1.0 / (1 << circ.n)
    kernels = []
    for v in range(len(doms)):
        K = np.zeros((N, N))
        for i, s in enumerate(states.tolist()):
            nb = []
            for u in range(doms[v]):
                t = list(s)
                t[v] = u
                nb.append(index[tuple(t)])
            w = weight[nb]
            tot = w.sum()
            if tot > 0:
                K[i, nb] += w / tot
            else:
                K[i, i] = 1.0
        kernels.append(K)
    for _ in range(sweeps):
        for K in kernels:
            dist = dist @ K
    return states, dist
