"""FP64 CPU oracle for multiple-testing correction of an all-pairs p matrix.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg may import this module.  It shares no code with the GPU
library and never imports it.

NApy (arXiv 2505.00448), Section 3.4: an output matrix may hold P-values
adjusted by Bonferroni, Benjamini-Hochberg or Benjamini-Yekutieli, and for a
matrix tested against itself the diagonal self-tests are not counted and are
NaN in every corrected matrix.

Readings (the paper does not spell these out):
  * The tests are the unordered pairs {i, j}, i != j: the symmetric matrix
    holds each test twice, and each is counted once (the upper triangle i < j
    is read and the result is written to both triangles).  The alternative
    reading would count both triangles, F (F - 1) tests, with every p-value
    duplicated.
  * A pair whose p-value is undefined (NaN) is not a performed test: it is left
    out of the count m and stays NaN.

Definitions, for the m defined p-values sorted ascending, p_(1) <= ... <= p_(m):
  * Bonferroni: p_adj = min(1, m p).
  * Benjamini-Hochberg (step-up): p_adj_(k) = min(1, min_{l >= k} m p_(l) / l).
  * Benjamini-Yekutieli: the same with m replaced by m c(m),
    c(m) = sum_{i=1}^{m} 1 / i.
Equal p-values receive equal adjusted values whatever their order in the sort
(the minimum over l >= k reaches the last of them).
"""

from __future__ import annotations

import math

import numpy as np

METHODS = ("bonferroni", "bh", "by")


def harmonic(m: int) -> float:
    """c(m) = sum_{i=1}^{m} 1/i, summed exactly then rounded once (math.fsum)."""
    return math.fsum(1.0 / i for i in range(1, m + 1))


def adjust_vector(p: np.ndarray, method: str) -> np.ndarray:
    """Adjusted p-values of a 1-D vector of defined (non-NaN) p-values."""
    p = np.asarray(p, dtype=np.float64)
    m = p.size
    if method not in METHODS:
        raise ValueError(method)
    if m == 0:
        return p.copy()
    if method == "bonferroni":
        return np.minimum(1.0, m * p)
    factor = float(m) if method == "bh" else m * harmonic(m)
    order = np.argsort(p, kind="stable")
    ps = p[order]
    k = np.arange(1, m + 1, dtype=np.float64)
    q = factor * ps / k
    # minimum over l >= k: a cumulative minimum from the right
    q = np.minimum.accumulate(q[::-1])[::-1]
    out = np.empty(m)
    out[order] = np.minimum(1.0, q)
    return out


def adjust_matrix(P: np.ndarray, method: str) -> np.ndarray:
    """Corrected copy of a symmetric F x F p matrix (reads the upper triangle)."""
    P = np.asarray(P, dtype=np.float64)
    F = P.shape[0]
    iu, ju = np.triu_indices(F, k=1)
    v = P[iu, ju]
    ok = ~np.isnan(v)
    adj = np.full(v.shape, np.nan)
    adj[ok] = adjust_vector(v[ok], method)
    out = np.full((F, F), np.nan)
    out[iu, ju] = adj
    out[ju, iu] = adj
    return out


def adjust_brute(p, method: str):
    """Tiny-input form in plain loops: the minimum over l >= k written out."""
    p = [float(x) for x in p]
    m = len(p)
    if method == "bonferroni":
        return [min(1.0, m * x) for x in p]
    factor = float(m) if method == "bh" else m * sum(1.0 / i for i in range(1, m + 1))
    ps = sorted(p)
    out = []
    for x in p:
        # rank of x: its first position in the sorted list; equal values reach
        # the same minimum from any of their positions
        k = ps.index(x) + 1
        out.append(min(1.0, min(factor * ps[l - 1] / l for l in range(k, m + 1))))
    return out
