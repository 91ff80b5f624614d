"""FP64 CPU oracle for the chi-squared test of independence between
categorical features with pairwise deletion.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg may import this module.  It shares no code with the GPU
library and never imports it.

NApy (arXiv 2505.00448):
  * Section 3.2: a pair (g, h) uses the samples I(g, h) where neither label is
    missing; Section 3.3: label-encoded categories (integers from 0);
    Section 3.4: for one matrix of F categorical features the outputs are
    F x F, entry (i, j) for features i and j.
  * Section 3.5 (chi-squared test): p from the survival function of the
    chi-squared distribution; if a category that exists in a feature becomes
    empty after the deletion, the statistic and every other output are NaN;
    if one of the two features has a single category, p and Cramer's V are NaN.
  * Table 2: the outputs are the chi-squared statistic, phi and Cramer's V
    (phi = V for a 2 x 2 table), and p.

Definitions: the r x c contingency table O of (g, h) on I(g, h), row sums
R_k, column sums C_l, N = |I|, E_kl = R_k C_l / N;
  chi2 = sum_kl (O_kl - E_kl)^2 / E_kl,  df = (r - 1)(c - 1),
  p = P(chi2_df > chi2),  V = sqrt(chi2 / (N min(r - 1, c - 1))).

Readings (the paper does not spell these out):
  * No continuity correction (Pearson's statistic; SciPy's chi2_contingency
    applies Yates' correction to 2 x 2 tables by default, correction=False
    matches).
  * The categories of a feature are the labels observed anywhere in its
    column; r and c count them.  With a single category the statistic is 0.
  * A column that is not label-encoded (a label that is not an integer,
    negative or at or above the caller's bound ncat) is not tested: NaN
    outputs and n = 0 for all its pairs.
  * The diagonal (g, g) is computed like any pair.
  * A pair without complete samples (N = 0) has no test: NaN outputs.
"""

from __future__ import annotations

from typing import Optional

import numpy as np
from scipy import stats


def table_test(O: np.ndarray):
    """(chi2, p, V) of an r x c table of counts whose rows and columns are the
    features' categories, with the paper's rules."""
    O = np.asarray(O, dtype=np.float64)
    r, c = O.shape
    R = O.sum(axis=1)
    C = O.sum(axis=0)
    N = O.sum()
    if np.any(R == 0) or np.any(C == 0) or N == 0:
        return np.nan, np.nan, np.nan
    E = np.outer(R, C) / N
    chi2 = float(np.sum((O - E) ** 2 / E))
    if r < 2 or c < 2:
        return chi2, np.nan, np.nan
    df = (r - 1) * (c - 1)
    p = float(stats.chi2.sf(chi2, df))
    V = float(np.sqrt(chi2 / (N * min(r - 1, c - 1))))
    return chi2, p, V


def chi2(L: np.ndarray, missing: Optional[float] = None, ncat: Optional[int] = None, pairs=None):
    """All pairs (or the listed (i, j) pairs) of the categorical columns of L
    (S x F float32): chi2, p, V (FP64) and n = |I|."""
    L = np.asarray(L, dtype=np.float32)
    S, F = L.shape
    miss = np.isnan(L)
    if missing is not None:
        miss |= L == np.float32(missing)
    cats = []
    for i in range(F):
        obs = L[~miss[:, i], i]
        ok = bool(np.all(obs == np.floor(obs)) and np.all(obs >= 0))
        if ok and ncat is not None and obs.size and obs.max() >= ncat:
            ok = False
        cats.append(np.unique(obs) if ok else None)
    full = pairs is None
    if full:
        pairs = [(i, j) for i in range(F) for j in range(F)]
    out = [np.full(len(pairs), np.nan) for _ in range(3)] + [np.zeros(len(pairs), dtype=np.int64)]
    for k, (i, j) in enumerate(pairs):
        if cats[i] is None or cats[j] is None:
            continue
        keep = ~miss[:, i] & ~miss[:, j]
        a, b = L[keep, i], L[keep, j]
        O = np.array([[np.sum((a == u) & (b == v)) for v in cats[j]] for u in cats[i]], dtype=np.float64)
        out[0][k], out[1][k], out[2][k] = table_test(O.reshape(len(cats[i]), len(cats[j])))
        out[3][k] = int(keep.sum())
    if full:
        return tuple(o.reshape(F, F) for o in out)
    return tuple(out)
