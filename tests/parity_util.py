"""Comparison rules shared by the GPU parity tests.

Counts are compared bit-exactly.  r within an absolute bound (1e-6 for the
FP32 / BF16x3 contractions, 1e-12 for the FP64 validation mode and for
Spearman, whose sums are exact integers).  NaN placement must match exactly.
P-values are compared through their conditioning: a p computed from an r that
is off by dr moves by |d ln p / dr| * dr in log space, with
    d ln p / dr = -2 sign(r) (1 - r^2)^(a-1) / (B(a, 1/2) p),  a = (n-2)/2,
so |ln p_gpu - ln p_oracle| <= 2 |d ln p/dr| dr_max + 1e-9 is required; where
the oracle's p underflows below 1e-300 the GPU's must be below 1e-290.
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
    from scipy import special
    p_gpu = np.asarray(p_gpu, dtype=np.float64).ravel()
    p_orc = np.asarray(p_orc, dtype=np.float64).ravel()
    r = np.asarray(r_orc, dtype=np.float64).ravel()
    n = np.asarray(n, dtype=np.int64).ravel()
    ng, no = np.isnan(p_gpu), np.isnan(p_orc)
    bad = np.flatnonzero(ng != no)
    assert bad.size == 0, f"{where}: p NaN placement differs at {bad.size} entries (first {bad[:5]})"
    ok = ~no
    tiny = ok & (p_orc < 1e-300)
    assert np.all(p_gpu[tiny] < 1e-290), f"{where}: underflowed p not reproduced"
    m = ok & ~tiny & (n >= 3)
    if not m.any():
        return
    a = (n[m] - 2) / 2.0
    rr = np.clip(np.abs(r[m]), 0, 1 - 1e-16)
    log_dp = np.log(2.0) + (a - 1) * np.log1p(-rr * rr) - special.betaln(a, 0.5) - np.log(p_orc[m])
    bound = 2.0 * np.exp(log_dp) * dr_max + 1e-9
    err = np.abs(np.log(np.maximum(p_gpu[m], 1e-320)) - np.log(p_orc[m]))
    worst = np.argmax(err - bound)
    assert np.all(err <= bound), (f"{where}: p off: |dlnp|={err[worst]:.3e} bound={bound[worst]:.3e} "
                                  f"p_gpu={p_gpu[m][worst]:.6e} p_orc={p_orc[m][worst]:.6e} n={n[m][worst]}")
    exact_one = ok & (n == 2)
    assert np.array_equal(p_gpu[exact_one], p_orc[exact_one]), f"{where}: p at n=2 differs"
