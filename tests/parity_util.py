"""Comparison rules shared by the GPU parity tests.

Counts are compared bit-exactly.  r within an absolute bound (1e-6 for the
FP32 / BF16x3 contractions, 1e-12 for the FP64 validation mode and for
Spearman, whose sums are exact integers).  NaN placement must match exactly.
P-values are compared through their conditioning: the GPU's p must lie
between the p-values of the oracle's |r| moved by twice the observed r error
either way (p is monotone in |r|), up to 1e-9 relative for the p routine
itself; this is the exact form of |d ln p| <= |d ln p / dr| |dr|.
"""

import numpy as np


def assert_counts_equal(n_gpu, n_orc, where=""):
    n_gpu = np.asarray(n_gpu, dtype=np.int64)
    n_orc = np.asarray(n_orc, dtype=np.int64)
    bad = np.argwhere(n_gpu != n_orc)
    assert bad.size == 0, f"{where}: {len(bad)} count mismatches, first at {bad[:5].tolist()}"


def assert_r_close(r_gpu, r_orc, tol, where=""):
    r_gpu = np.asarray(r_gpu, dtype=np.float64)
    r_orc = np.asarray(r_orc, dtype=np.float64)
    ng, no = np.isnan(r_gpu), np.isnan(r_orc)
    bad = np.argwhere(ng != no)
    assert bad.size == 0, (f"{where}: NaN placement differs at {len(bad)} entries, first "
                           f"{bad[:5].tolist()} gpu={r_gpu[tuple(bad[0])] if bad.size else None} "
                           f"orc={r_orc[tuple(bad[0])] if bad.size else None}")
    ok = ~no
    if ok.any():
        err = np.abs(r_gpu[ok] - r_orc[ok])
        worst = float(err.max())
        assert worst <= tol, f"{where}: max |dr| = {worst:.3e} > {tol:.1e}"
        return worst
    return 0.0


def assert_p_close(p_gpu, p_orc, r_orc, n, dr_max, where=""):
    """p = I_{1-r^2}((n-2)/2, 1/2) falls monotonically in |r|, so an r that
    is within d of the oracle's gives a p between the values at |r| + d and
    |r| - d (d = 2 dr_max plus rounding); 1e-9 relative slack covers the
    p routine's own error.  n = 2 (Pearson p = 1) must match exactly."""
    from oracle.oracle import beta_tail
    p_gpu = np.asarray(p_gpu, dtype=np.float64).ravel()
    p_orc = np.asarray(p_orc, dtype=np.float64).ravel()
    r = np.asarray(r_orc, dtype=np.float64).ravel()
    n = np.asarray(n, dtype=np.int64).ravel()
    ng, no = np.isnan(p_gpu), np.isnan(p_orc)
    bad = np.flatnonzero(ng != no)
    assert bad.size == 0, f"{where}: p NaN placement differs at {bad.size} entries (first {bad[:5]})"
    ok = ~no
    two = ok & (n == 2)
    assert np.array_equal(p_gpu[two], p_orc[two]), f"{where}: p at n=2 differs"
    m = ok & (n >= 3)
    if not m.any():
        return
    d = 2.0 * dr_max + 4e-16
    a = (n[m] - 2) / 2.0
    ar = np.abs(r[m])
    r_hi = np.clip(ar + d, 0.0, 1.0)
    r_lo = np.clip(ar - d, 0.0, 1.0)
    p_min = beta_tail(a, r_hi)
    p_max = beta_tail(a, r_lo)
    pg = p_gpu[m]
    ok_lo = pg >= p_min * (1 - 1e-9) - 1e-300
    ok_hi = pg <= p_max * (1 + 1e-9) + 1e-300
    good = ok_lo & ok_hi
    if not good.all():
        w = int(np.flatnonzero(~good)[0])
        raise AssertionError(f"{where}: p_gpu={pg[w]:.6e} outside [{p_min[w]:.6e}, {p_max[w]:.6e}] "
                             f"(p_orc={p_orc[m][w]:.6e}, r={r[m][w]!r}, n={n[m][w]})")
