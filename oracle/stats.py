"""Sampling-accuracy statistics (Sec. 3.3.3) for the oracle.

Test infrastructure only (see ``oracle/__init__.py``).

Sec. 3.3.3 measures sampled-versus-exact distributions with the KL
divergence; the tests here add Pearson's chi-square goodness of fit, with
bins whose expected count is below 5 pooled into one bin.
"""
from __future__ import annotations

import numpy as np
from scipy import stats as _st


def chi2_pooled(counts, probs, min_expected=5.0):
    """Pearson chi-square of observed counts against probabilities.
    Returns (statistic, dof, p_value)."""
    counts = np.asarray(counts, dtype=np.float64)
    probs = np.asarray(probs, dtype=np.float64)
    probs = probs / probs.sum()
    n = counts.sum()
    exp = n * probs
    big = exp >= min_expected
    obs_b, exp_b = list(counts[big]), list(exp[big])
    rest_o, rest_e = counts[~big].sum(), exp[~big].sum()
    if rest_e > 0:
        obs_b.append(rest_o)
        exp_b.append(rest_e)
    obs_b, exp_b = np.array(obs_b), np.array(exp_b)
    stat = float(np.sum((obs_b - exp_b) ** 2 / exp_b))
    dof = max(1, len(obs_b) - 1)
    return stat, dof, float(_st.chi2.sf(stat, dof))


def kl_divergence(counts, probs):
    """KL(empirical || exact); empty bins contribute nothing."""
    counts = np.asarray(counts, dtype=np.float64)
    q = counts / counts.sum()
    p = np.asarray(probs, dtype=np.float64)
    m = q > 0
    return float(np.sum(q[m] * np.log(q[m] / p[m])))


def uniformity_pvalue(pvals):
    """Kolmogorov-Smirnov p-value of a sample of p-values against U(0,1)."""
    return float(_st.kstest(np.asarray(pvals), "uniform").pvalue)
