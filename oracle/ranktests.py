"""FP64 CPU oracle for the rank tests of categorical x continuous pairs with
pairwise deletion: Mann-Whitney U (dichotomous) and Kruskal-Wallis H
(categorical).

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg may import this module.  It shares no code with the GPU
library and never imports it.

NApy (arXiv 2505.00448), Section 3.5:
  * Mann-Whitney U: ranks of the continuous values within I(g, h), ties given
    their average rank; the z-value uses the usual tie correction; p exact or
    asymptotic (survival function of the standard normal); in the automatic
    mode exact when the pair has no ties and one of the two groups has fewer
    than eight samples, else asymptotic; NaN when a group is empty.
  * Kruskal-Wallis H: average ranks, tie-corrected H, p from the survival
    function of the chi-squared distribution (K - 1 degrees of freedom); NaN
    when a category of the feature is empty within I(g, h).

Definitions (n = |I|, groups by label, R_k the rank sum of group k, T =
sum over tie runs of t^3 - t):
  * U1 = R_0 - n_0 (n_0 + 1) / 2 (group of label 0 first: the statistic of
    scipy.stats.mannwhitneyu(group0, group1)); U2 = n_0 n_1 - U1.
  * asymptotic two-sided p: U = max(U1, U2), mu = n_0 n_1 / 2,
    s^2 = n_0 n_1 / 12 ((n + 1) - T / (n (n - 1))),
    z = (U - mu - 1/2) / s (continuity correction), p = min(1, 2 sf(z)).
  * exact two-sided p: p = min(1, 2 P(U' >= max(U1, U2))) with U' the
    statistic of a random split, counted from the generating function
    prod_{i=1}^{m} (1 - q^(M+i)) / (1 - q^i) (m, M the group sizes).
  * H = (12 / (n (n + 1)) sum_k R_k^2 / n_k - 3 (n + 1)) / (1 - T / (n^3 - n)),
    p = P(chi2_{K-1} > H).

Readings (the paper does not spell these out):
  * MWU groups: labels 0 and 1; other labels make the column untested (NaN,
    n = 0), as for the t-test.  The continuity correction is applied (SciPy's
    default).  All values tied within I: s = 0, z = -inf, p = 1.
  * Kruskal-Wallis categories: the labels observed anywhere in the column;
    one category, or all values tied within I (the correction's denominator
    is 0), gives NaN.
"""

from __future__ import annotations

from typing import Optional

import numpy as np
from scipy import special, stats


def _ranks_and_ties(y: np.ndarray):
    r = stats.rankdata(y, method="average")
    _, counts = np.unique(y, return_counts=True)
    T = float(np.sum(counts.astype(np.float64) ** 3 - counts))
    return r, T


def mwu_exact_sf(u: int, m: int, M: int) -> float:
    """P(U' >= u) for a random split into groups of m and M without ties, from
    the generating function's coefficients (counts of arrangements by U')."""
    D = m * M
    c = np.zeros(D + 1)
    c[0] = 1.0
    for i in range(1, min(m, M) + 1):
        big = max(m, M)
        # multiply by (1 - q^(big + i)), then divide by (1 - q^i)
        c[big + i:] -= c[: D + 1 - (big + i)].copy()
        for d in range(i, D + 1):
            c[d] += c[d - i]
    total = c.sum()
    return float(c[u:].sum() / total) if u <= D else 0.0


def mwu_pair(y0: np.ndarray, y1: np.ndarray, mode: str = "auto"):
    """(U1, p) with the paper's rules; mode 'auto' or 'asymptotic'."""
    n0, n1 = y0.size, y1.size
    if n0 == 0 or n1 == 0:
        return np.nan, np.nan
    r, T = _ranks_and_ties(np.concatenate([y0, y1]))
    n = n0 + n1
    R0 = float(r[:n0].sum())
    U1 = R0 - n0 * (n0 + 1) / 2.0
    U2 = n0 * n1 - U1
    U = max(U1, U2)
    exact = mode == "auto" and T == 0.0 and min(n0, n1) < 8
    if exact:
        p = 2.0 * mwu_exact_sf(int(round(U)), n0, n1)
    else:
        s2 = n0 * n1 / 12.0 * ((n + 1) - T / (n * (n - 1))) if n > 1 else 0.0
        s = np.sqrt(s2)
        z = (U - n0 * n1 / 2.0 - 0.5) / s if s > 0 else -np.inf
        p = 2.0 * stats.norm.sf(z)
    return float(U1), float(min(1.0, p))


def kruskal_groups(groups):
    """(H, p) for a list of FP64 arrays, with the paper's rules."""
    K = len(groups)
    if K < 2 or any(g.size == 0 for g in groups):
        return np.nan, np.nan
    allv = np.concatenate(groups)
    n = allv.size
    r, T = _ranks_and_ties(allv)
    denom = 1.0 - T / (float(n) ** 3 - n)
    if denom <= 0.0:
        return np.nan, np.nan
    pos = np.cumsum([0] + [g.size for g in groups])
    s = sum(float(r[pos[k]:pos[k + 1]].sum()) ** 2 / groups[k].size for k in range(K))
    H = (12.0 / (n * (n + 1.0)) * s - 3.0 * (n + 1.0)) / denom
    return float(H), float(special.chdtrc(K - 1, H))


def _run(L, X, missing, pairs, test, dichotomous, ncat):
    L = np.asarray(L, dtype=np.float32)
    X = np.asarray(X, dtype=np.float32)
    S, FC = L.shape
    FQ = X.shape[1]
    mL = np.isnan(L)
    mX = np.isnan(X)
    if missing is not None:
        mL |= L == np.float32(missing)
        mX |= X == np.float32(missing)
    cats = []
    for i in range(FC):
        obs = L[~mL[:, i], i]
        ok = bool(np.all(obs == np.floor(obs)) and np.all(obs >= 0))
        if ok and ncat is not None and obs.size and obs.max() >= ncat:
            ok = False
        if ok and dichotomous and not np.all(np.isin(obs, [0.0, 1.0])):
            ok = False
        cats.append((np.array([0.0, 1.0]) if dichotomous else np.unique(obs)) if ok else None)
    full = pairs is None
    if full:
        pairs = [(i, j) for i in range(FC) for j in range(FQ)]
    st = np.full(len(pairs), np.nan)
    pv = np.full(len(pairs), np.nan)
    nn = np.zeros(len(pairs), dtype=np.int64)
    for k, (i, j) in enumerate(pairs):
        if cats[i] is None:
            continue
        keep = ~mL[:, i] & ~mX[:, j]
        lab = L[keep, i]
        y = X[keep, j].astype(np.float64)
        st[k], pv[k] = test([y[lab == c] for c in cats[i]])
        nn[k] = int(keep.sum())
    if full:
        return st.reshape(FC, FQ), pv.reshape(FC, FQ), nn.reshape(FC, FQ)
    return st, pv, nn


def mannwhitney(L, X, mode: str = "auto", missing: Optional[float] = None, pairs=None):
    """All pairs (or the listed pairs) of dichotomous columns of L and
    continuous columns of X: U (of the label-0 group), p, n."""
    return _run(L, X, missing, pairs, lambda gs: mwu_pair(gs[0], gs[1], mode), True, None)


def kruskal(L, X, missing: Optional[float] = None, pairs=None, ncat: Optional[int] = None):
    return _run(L, X, missing, pairs, kruskal_groups, False, ncat)
