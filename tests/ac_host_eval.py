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
