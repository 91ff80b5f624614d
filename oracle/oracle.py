"""FP64 CPU oracle: Python driver around napy_oracle.c plus the p-values.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg may import this module.  It shares no code with the GPU
library and never imports it.

P-values (NApy, arXiv 2505.00448):
  * Section 3.5.2 gives Pearson's two-sided p from the CDF of the Beta
    distribution; Section 3.5.3 gives Spearman's from the t distribution.
    Under the null, r on [-1, 1] follows a Beta(n/2 - 1, n/2 - 1) law, and the
    two-sided tail equals the regularized incomplete beta function
    I_{1-r^2}((n-2)/2, 1/2); with df = n - 2 and t = r sqrt(df / (1 - r^2))
    this is exactly the two-sided Student-t tail, so both sections reduce to
    the same function.  ``scipy.special.betainc`` evaluates it.
  * Pearson p is undefined for fewer than two pairwise-complete samples
    (Section 3.5.2), so at n = 2 it is defined; its value there is the limit
    of I_x(a, 1/2) as a -> 0, i.e. 1 (reading, matching SciPy).
  * Spearman p is undefined for n <= 2 (Section 3.5.3).
"""

from __future__ import annotations

import ctypes
import math
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "napy_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

# Reading of Section 3.5.2: the value of Pearson's p at exactly two
# pairwise-complete samples.  The alternative reading would be NaN.
PEARSON_P_AT_N2 = 1.0

_lib = None


def build(force: bool = False) -> str:
    """Compile napy_oracle.c with gcc/OpenMP into oracle/liboracle.so."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared",
                               "-std=c11", "-Wall", "-Werror", "-fno-fast-math",
                               "-ffp-contract=off",
                               _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        i64 = ctypes.c_int64
        lib.orc_all_pairs.argtypes = [P, i64, i64, i64, ctypes.c_int, ctypes.c_double,
                                      ctypes.c_int, ctypes.c_int, P, P]
        lib.orc_all_pairs.restype = ctypes.c_int
        lib.orc_pairs.argtypes = [P, i64, i64, i64, ctypes.c_int, ctypes.c_double,
                                  ctypes.c_int, ctypes.c_int, P, P, i64, P, P]
        lib.orc_pairs.restype = ctypes.c_int
        lib.orc_pair_ranks.argtypes = [P, i64, i64, i64, i64, ctypes.c_int, ctypes.c_double, P, P]
        lib.orc_pair_ranks.restype = i64
        lib.orc_max_threads.argtypes = []
        lib.orc_max_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def max_threads() -> int:
    return int(_load().orc_max_threads())


def _prep(X: np.ndarray) -> np.ndarray:
    X = np.asarray(X)
    if X.ndim != 2:
        raise ValueError("X must be samples x variables")
    return np.ascontiguousarray(X, dtype=np.float64)


def _sentinel(missing: Optional[float]):
    if missing is None or (isinstance(missing, float) and math.isnan(missing)):
        return 0, 0.0
    return 1, float(missing)


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def corr_all(X: np.ndarray, method: str, missing: Optional[float] = None,
             nthreads: int = 0):
    """All pairs (both triangles and the diagonal): returns (r, n) with r
    float64 [F, F] and n int64 [F, F]."""
    lib = _load()
    Xd = _prep(X)
    S, F = Xd.shape
    r = np.empty((F, F), dtype=np.float64)
    n = np.empty((F, F), dtype=np.int64)
    us, sv = _sentinel(missing)
    rc = lib.orc_all_pairs(_ptr(Xd), S, F, F, us, sv, int(method == "spearman"),
                           int(nthreads), _ptr(r), _ptr(n))
    if rc != 0:
        raise MemoryError("oracle buffer allocation failed")
    return r, n


def corr_pairs(X: np.ndarray, gi, hi, method: str, missing: Optional[float] = None,
               nthreads: int = 0):
    """Listed pairs: returns (r, n) with one entry per (gi[k], hi[k])."""
    lib = _load()
    Xd = _prep(X)
    S, F = Xd.shape
    g = np.ascontiguousarray(gi, dtype=np.int64)
    h = np.ascontiguousarray(hi, dtype=np.int64)
    if g.shape != h.shape or g.ndim != 1:
        raise ValueError("pair index arrays must be 1-D and of equal length")
    if g.size and (g.min() < 0 or h.min() < 0 or g.max() >= F or h.max() >= F):
        raise ValueError("pair index out of range")
    r = np.empty(g.size, dtype=np.float64)
    n = np.empty(g.size, dtype=np.int64)
    us, sv = _sentinel(missing)
    rc = lib.orc_pairs(_ptr(Xd), S, F, F, us, sv, int(method == "spearman"), int(nthreads),
                       _ptr(g), _ptr(h), g.size, _ptr(r), _ptr(n))
    if rc != 0:
        raise MemoryError("oracle buffer allocation failed")
    return r, n


def pair_ranks(X: np.ndarray, g: int, h: int, missing: Optional[float] = None):
    """Average ranks inside I(g,h) for both sides, in sample order, NaN for
    samples outside I(g,h).  Returns (rank_g, rank_h, n)."""
    lib = _load()
    Xd = _prep(X)
    S, F = Xd.shape
    if not (0 <= g < F and 0 <= h < F):
        raise ValueError("variable index out of range")
    rg = np.empty(S, dtype=np.float64)
    rh = np.empty(S, dtype=np.float64)
    us, sv = _sentinel(missing)
    n = lib.orc_pair_ranks(_ptr(Xd), S, F, g, h, us, sv, _ptr(rg), _ptr(rh))
    if n < 0:
        raise MemoryError("oracle buffer allocation failed")
    return rg, rh, int(n)


def beta_tail(a, ar) -> np.ndarray:
    """I_{1-r^2}(a, 1/2) for |r| = ar in [0, 1], through scipy's betainc.

    1 - r^2 rounds to 1 in FP64 once r^2 is below the machine epsilon, which
    would give p = 1 where the true p is 1 - O(|r| sqrt(a)).  So where p > 1/2
    the same quantity is taken through the symmetry I_x(a, b) = 1 - I_{1-x}(b, a)
    as 1 - I_{r^2}(1/2, a), and elsewhere directly.  There 1 - r^2 is formed
    as 1 - r*r for |r| < 1/2 (within an ulp of 1) and as (1 - |r|)(1 + |r|)
    above, where 1 - |r| is exact: p at large a amplifies a relative error of
    1 - r^2 about a-fold."""
    from scipy import special
    a = np.asarray(a, dtype=np.float64)
    ar = np.clip(np.abs(np.asarray(ar, dtype=np.float64)), 0.0, 1.0)
    x = np.where(ar < 0.5, 1.0 - ar * ar, (1.0 - ar) * (1.0 + ar))
    direct = special.betainc(a, 0.5, x)
    comp = 1.0 - special.betainc(0.5, a, ar * ar)
    return np.where(comp > 0.5, comp, direct)


def pvalue(r, n, method: str) -> np.ndarray:
    """Two-sided p = I_{1-r^2}((n-2)/2, 1/2) with the paper's undefined cases."""
    r = np.asarray(r, dtype=np.float64)
    n = np.asarray(n, dtype=np.int64)
    p = np.full(np.broadcast(r, n).shape, np.nan, dtype=np.float64)
    r_b = np.broadcast_to(r, p.shape)
    n_b = np.broadcast_to(n, p.shape)
    ok = (n_b >= 3) & np.isfinite(r_b)
    a = (n_b[ok] - 2).astype(np.float64) / 2.0
    p[ok] = beta_tail(a, r_b[ok])
    if method == "pearson":
        two = (n_b == 2) & np.isfinite(r_b)
        p[two] = PEARSON_P_AT_N2
    return p


def pvalue_mp(r: float, n: int, dps: int = 50) -> float:
    """The same p in arbitrary precision (mpmath), for pins."""
    import mpmath
    with mpmath.workdps(dps):
        a = mpmath.mpf(int(n) - 2) / 2
        y = mpmath.mpf(float(r)) ** 2
        # the same value through I_x(a, b) = 1 - I_{1-x}(b, a) while that keeps
        # at least half of the working digits: mpmath's series for I_x(a, 1/2)
        # stalls for x near 1 and large a
        comp = 1 - mpmath.betainc(mpmath.mpf(1) / 2, a, 0, y, regularized=True)
        if comp > mpmath.mpf(10) ** (-(dps // 2)):
            return float(comp)
        return float(mpmath.betainc(a, mpmath.mpf(1) / 2, 0, 1 - y, regularized=True))


def pearson(X: np.ndarray, missing: Optional[float] = None, nthreads: int = 0):
    """Oracle Pearson: (r float64 [F,F], p float64 [F,F], n int64 [F,F])."""
    r, n = corr_all(X, "pearson", missing, nthreads)
    return r, pvalue(r, n, "pearson"), n


def spearman(X: np.ndarray, missing: Optional[float] = None, nthreads: int = 0):
    """Oracle Spearman: (rho float64 [F,F], p float64 [F,F], n int64 [F,F])."""
    r, n = corr_all(X, "spearman", missing, nthreads)
    return r, pvalue(r, n, "spearman"), n


def pearson_pairs(X, gi, hi, missing=None, nthreads: int = 0):
    r, n = corr_pairs(X, gi, hi, "pearson", missing, nthreads)
    return r, pvalue(r, n, "pearson"), n


def spearman_pairs(X, gi, hi, missing=None, nthreads: int = 0):
    r, n = corr_pairs(X, gi, hi, "spearman", missing, nthreads)
    return r, pvalue(r, n, "spearman"), n
