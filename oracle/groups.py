"""FP64 CPU oracle for the categorical x continuous tests with pairwise
deletion: two-sample t-test (Student or Welch) and one-way ANOVA.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg may import this module.  It shares no code with the GPU
library and never imports it.

NApy (arXiv 2505.00448):
  * Section 3.2: a pair (g, h) uses the samples I(g, h) where neither value is
    missing.  Section 3.3: categorical features are label-encoded (integers
    from 0).  Section 3.4: for F_C categorical and F_Q continuous features the
    outputs are F_C x F_Q matrices, entry (i, j) for categorical feature i and
    continuous feature j.
  * Section 3.5 (t-test): Student's or Welch's two-sample t; two-sided p from
    the t distribution's survival function; undefined (NaN) when a group has
    fewer than two samples or both together fewer than three, and for
    Student's test when the pooled standard deviation is zero.
  * Section 3.5 (ANOVA): F from the two sums of squares; p from the survival
    function of Fisher's F distribution; undefined when a category is empty
    after the deletion; when every within-category variance is zero, F = inf
    and p = 0 unless all category means are equal, then NaN.

Readings (the paper does not spell these out):
  * t-test groups: label 0 and label 1; t = (mean_0 - mean_1) / se, the sign
    of scipy.stats.ttest_ind(group0, group1).  A column with any other label
    is not dichotomous: its results are NaN.
  * Welch with both group variances zero: t = +-inf, p = 0 when the means
    differ, NaN when they are equal (the rule the paper states for ANOVA; the
    paper only says Cohen's D is undefined there).
  * ANOVA categories of a column: the distinct labels observed anywhere in the
    column; "empty" is checked for each of them within I(g, h).  A column with
    a single category has no F (NaN).
  * "All category means equal" (the paper says group sums) for the
    zero-variance rule.
  * Zero variance is exact: every value of the group is equal (minimum ==
    maximum), not a computed variance below a threshold.
  * A column that is not label-encoded as the test needs (a label that is not
    an integer, negative, at or above the caller's category bound, or for the
    t-test not 0 or 1) is not tested: its statistics and p-values are NaN and
    its counts 0.
"""

from __future__ import annotations

from typing import Optional

import numpy as np
from scipy import stats


def _missing(v: np.ndarray, sentinel: Optional[float]) -> np.ndarray:
    m = np.isnan(v)
    if sentinel is not None:
        m |= v == np.float32(sentinel)
    return m


def _labels(col: np.ndarray, miss: np.ndarray):
    """Integer labels of a column and whether all observed labels are integers >= 0."""
    obs = col[~miss]
    ok = bool(np.all(obs == np.floor(obs)) and np.all(obs >= 0))
    return col, ok


def ttest_pair(y0: np.ndarray, y1: np.ndarray, welch: bool):
    """(t, p) for two groups of FP64 values, with the paper's rules."""
    n0, n1 = y0.size, y1.size
    if n0 < 2 or n1 < 2 or n0 + n1 < 3:
        return np.nan, np.nan
    m0, m1 = y0.mean(), y1.mean()
    ss0 = float(np.sum((y0 - m0) ** 2))
    ss1 = float(np.sum((y1 - m1) ** 2))
    const0 = y0.min() == y0.max()
    const1 = y1.min() == y1.max()
    d = m0 - m1
    if not welch:
        if const0 and const1:  # pooled standard deviation zero
            return np.nan, np.nan
        df = n0 + n1 - 2
        sp2 = (ss0 + ss1) / df
        t = d / np.sqrt(sp2 * (1.0 / n0 + 1.0 / n1))
    else:
        if const0 and const1:
            if d == 0.0:
                return np.nan, np.nan
            return float(np.copysign(np.inf, d)), 0.0
        v0 = ss0 / (n0 - 1) / n0
        v1 = ss1 / (n1 - 1) / n1
        t = d / np.sqrt(v0 + v1)
        df = (v0 + v1) ** 2 / (v0 * v0 / (n0 - 1) + v1 * v1 / (n1 - 1))
    p = 2.0 * stats.t.sf(abs(t), df)
    return float(t), float(p)


def anova_groups(groups):
    """(F, p) for a list of FP64 arrays (the categories of one column within
    I(g, h)), with the paper's rules."""
    K = len(groups)
    if K < 2 or any(g.size == 0 for g in groups):
        return np.nan, np.nan
    N = sum(g.size for g in groups)
    means = [g.mean() for g in groups]
    allc = np.concatenate(groups)
    grand = allc.mean()
    ssb = float(sum(g.size * (mk - grand) ** 2 for g, mk in zip(groups, means)))
    ssw = float(sum(np.sum((g - mk) ** 2) for g, mk in zip(groups, means)))
    if all(g.min() == g.max() for g in groups):  # every within-category variance zero
        if all(mk == means[0] for mk in means):
            return np.nan, np.nan
        return np.inf, 0.0
    df1, df2 = K - 1, N - K
    F = (ssb / df1) / (ssw / df2)
    return float(F), float(stats.f.sf(F, df1, df2))


def ttest(L: np.ndarray, X: np.ndarray, welch: bool = False, missing: Optional[float] = None,
          pairs=None):
    """All pairs (or the listed (i, j) pairs) of categorical columns of L and
    continuous columns of X (both S x F, float32): t, p (FP64) and n = |I|."""
    return _run(L, X, missing, pairs, lambda gs: ttest_pair(gs[0], gs[1], welch) if len(gs) == 2 else (np.nan, np.nan),
                dichotomous=True)


def anova(L: np.ndarray, X: np.ndarray, missing: Optional[float] = None, pairs=None,
          ncat: Optional[int] = None):
    """ncat: labels must lie in [0, ncat) (no bound if None)."""
    return _run(L, X, missing, pairs, anova_groups, dichotomous=False, ncat=ncat)


def _run(L, X, missing, pairs, test, dichotomous: bool, ncat: Optional[int] = None):
    L = np.asarray(L, dtype=np.float32)
    X = np.asarray(X, dtype=np.float32)
    S, FC = L.shape
    FQ = X.shape[1]
    mL = _missing(L, missing)
    mX = _missing(X, missing)
    cats = []
    for i in range(FC):
        col, ok = _labels(L[:, i], mL[:, i])
        labs = np.unique(col[~mL[:, i]]) if ok else None
        if dichotomous and labs is not None and not np.all(np.isin(labs, [0.0, 1.0])):
            labs = None
        if ncat is not None and labs is not None and labs.size and labs.max() >= ncat:
            labs = None
        if dichotomous and labs is not None:
            labs = np.array([0.0, 1.0])  # both groups are required
        cats.append(labs)
    if pairs is None:
        pairs = [(i, j) for i in range(FC) for j in range(FQ)]
        stat = np.full((FC, FQ), np.nan)
        pv = np.full((FC, FQ), np.nan)
        nn = np.zeros((FC, FQ), dtype=np.int64)
        put = lambda k, i, j, s, p, n: (stat.__setitem__((i, j), s), pv.__setitem__((i, j), p),
                                        nn.__setitem__((i, j), n))
    else:
        stat = np.full(len(pairs), np.nan)
        pv = np.full(len(pairs), np.nan)
        nn = np.zeros(len(pairs), dtype=np.int64)
        put = lambda k, i, j, s, p, n: (stat.__setitem__(k, s), pv.__setitem__(k, p), nn.__setitem__(k, n))
    for k, (i, j) in enumerate(pairs):
        keep = ~mL[:, i] & ~mX[:, j]
        n = int(keep.sum())
        labs = cats[i]
        if labs is None:
            put(k, i, j, np.nan, np.nan, 0)
            continue
        lab = L[keep, i]
        y = X[keep, j].astype(np.float64)
        groups = [y[lab == c] for c in labs]
        s, p = test(groups)
        put(k, i, j, s, p, n)
    return stat, pv, nn
