"""Host-side reading of a compiled AC, for checking the compiler on the CPU.

Test helper only: it evaluates the flat DAG that the compiler produced (with
arbitrary complex indicator values, which is what the polynomial-identity
test needs).  The GPU library never uses it.
"""
import numpy as np

from paper_2103_17226_amd.compiler import IND_VAL_SHIFT, NO_SLOT, TAG_IND, TAG_NODE, TAG_SEL, TAG_SHIFT


def slot_values(ac, theta, noise=None):
    noise = ac.noise_default if noise is None else noise
    return np.array([s.value(theta, noise) for s in ac.slots], dtype=np.complex128)


def evaluate(ac, theta, lam, noise=None):
    """lam[v][u] = complex indicator value; returns the root value."""
    W = slot_values(ac, theta, noise)
    val = np.zeros(ac.n_internal, dtype=np.complex128)
    mask = (1 << TAG_SHIFT) - 1
    for i in range(ac.n_internal):
        kids = []
        for r in ac.col[ac.row_ptr[i]:ac.row_ptr[i + 1]]:
            r = int(r)
            tag, x = r >> TAG_SHIFT, r & mask
            if tag == TAG_NODE:
                kids.append(val[x])
            elif tag == TAG_IND:
                kids.append(lam[x & ((1 << IND_VAL_SHIFT) - 1)][x >> IND_VAL_SHIFT])
            elif tag == TAG_SEL:
                v, sl = ac.selectors[x]
                kids.append(sum(lam[v][u] * (0 if s == NO_SLOT else W[s]) for u, s in enumerate(sl)))
            else:
                kids.append(W[x])
        val[i] = np.sum(kids) if ac.op[i] == 0 else np.prod(kids)
    return val[ac.root]


def evaluate_assignment(ac, theta, values, noise=None):
    lam = []
    for v, d in enumerate(ac.var_dom):
        row = np.zeros(d, dtype=np.complex128)
        row[int(values[v])] = 1.0
        lam.append(row)
    return evaluate(ac, theta, lam, noise)


def max_product(ac, theta, x_bits, noise=None):
    """Most probable noise events for outcome x on an AC compiled for it:
    nodes with an event indicator below hold M = max over those events of
    |value|^2 (products multiply, sums take the largest branch), the others
    complex values; event indicators are 1, output indicators follow x.
    Returns (M at the root, the event values along the largest branches
    (first largest in child order), None for events not met)."""
    W = slot_values(ac, theta, noise)
    n = ac.n_qubits
    mask = (1 << TAG_SHIFT) - 1
    vmask = (1 << IND_VAL_SHIFT) - 1
    val = np.zeros(ac.n_internal, dtype=np.complex128)
    big = np.zeros(ac.n_internal, dtype=bool)          # an event indicator below
    M = np.zeros(ac.n_internal)

    def kid(r):
        """(is max-domain, M or complex value) of a child reference."""
        tag, x = r >> TAG_SHIFT, r & mask
        if tag == TAG_NODE:
            return (True, M[x]) if big[x] else (False, val[x])
        if tag == TAG_IND:
            v, u = x & vmask, x >> IND_VAL_SHIFT
            if v >= n:
                return True, 1.0
            return False, complex(1.0 if int(x_bits[v]) == u else 0.0)
        if tag == TAG_SEL:
            raise ValueError("selector leaves hide the noise events")
        return False, W[x]

    for i in range(ac.n_internal):
        ks = [kid(int(r)) for r in ac.col[ac.row_ptr[i]:ac.row_ptr[i + 1]]]
        big[i] = any(b for b, _ in ks)
        if not big[i]:
            vals = [v for _, v in ks]
            val[i] = np.sum(vals) if ac.op[i] == 0 else np.prod(vals)
            continue
        ms = [v if b else abs(v) ** 2 for b, v in ks]
        M[i] = max(ms) if ac.op[i] == 0 else float(np.prod(ms))
    r = ac.root
    if not big[r]:
        return abs(val[r]) ** 2, [None] * (len(ac.var_dom) - n)
    k = [None] * (len(ac.var_dom) - n)
    sel = np.zeros(ac.n_internal, dtype=bool)
    sel[r] = True
    for i in range(ac.n_internal - 1, -1, -1):
        if not (sel[i] and big[i]):
            continue
        refs = [int(x) for x in ac.col[ac.row_ptr[i]:ac.row_ptr[i + 1]]]
        if ac.op[i] == 0:
            ms = [(v if b else abs(v) ** 2) for b, v in (kid(x) for x in refs)]
            refs = [refs[int(np.argmax(ms))]]
        for x in refs:
            tag, y = x >> TAG_SHIFT, x & mask
            if tag == TAG_NODE and big[y]:
                sel[y] = True
            elif tag == TAG_IND and (y & vmask) >= n:
                k[(y & vmask) - n] = y >> IND_VAL_SHIFT
    return M[r], k
