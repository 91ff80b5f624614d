"""Pins of the FP64 oracle against facts fixed by the paper's definitions and
by mathematics, never against itself.

Definitions: pairwise-complete set (Section 3.2), Pearson with its undefined
cases (Section 3.5.2), Spearman with average ranks inside the pair subset and
its undefined cases (Section 3.5.3), p = I_{1-r^2}((n-2)/2, 1/2).
"""

import itertools
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

from oracle import oracle as orc
from oracle import grad as ograd
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "edge_cases.json")


# --------------------------------------------------------------------------
# golden, hand-derived edge cases
# --------------------------------------------------------------------------

def test_golden_edge_cases():
    X = synth.edge_matrix()
    with open(GOLDEN) as f:
        cases = json.load(f)["cases"]
    outs = {m: (orc.pearson(X) if m == "pearson" else orc.spearman(X)) for m in ("pearson", "spearman")}
    for c in cases:
        r, p, n = outs[c["method"]]
        g, h = c["g"], c["h"]
        assert n[g, h] == c["n"] and n[h, g] == c["n"], c
        if c["r"] is None:
            assert math.isnan(r[g, h]), c
        else:
            assert abs(r[g, h] - c["r"]) <= 1e-14, (c, r[g, h])
        if c["p"] is None:
            assert math.isnan(p[g, h]), c
        elif c["p"] == "mp":
            ref = orc.pvalue_mp(c["r"], c["n"])
            assert abs(p[g, h] - ref) <= 1e-13 * max(ref, 1e-300), (c, p[g, h], ref)
        else:
            assert abs(p[g, h] - c["p"]) <= 1e-14, (c, p[g, h])


# --------------------------------------------------------------------------
# brute force with exact rational arithmetic on tiny inputs
# --------------------------------------------------------------------------

def _exact_r2_and_sign(a, b):
    """Exact r^2 and the sign of the covariance from rationals."""
    n = len(a)
    A = [Fraction(float(v)) for v in a]
    B = [Fraction(float(v)) for v in b]
    ma = sum(A) / n
    mb = sum(B) / n
    sab = sum((x - ma) * (y - mb) for x, y in zip(A, B))
    saa = sum((x - ma) ** 2 for x in A)
    sbb = sum((y - mb) ** 2 for y in B)
    if saa == 0 or sbb == 0:
        return None, 0
    return sab * sab / (saa * sbb), (sab > 0) - (sab < 0)


def _exact_avg_ranks(v):
    """Average ranks by direct counting: rank = #less + (#equal + 1) / 2."""
    out = []
    for x in v:
        less = sum(1 for y in v if y < x)
        eq = sum(1 for y in v if y == x)
        out.append(Fraction(2 * less + eq + 1, 2))
    return out


def test_bruteforce_exact_tiny():
    rng = np.random.default_rng(11)
    for trial in range(60):
        S = int(rng.integers(1, 9))
        F = int(rng.integers(1, 5))
        X = rng.integers(-3, 4, size=(S, F)).astype(np.float32)
        if trial % 2:
            X = (X + rng.standard_normal((S, F)).astype(np.float32)).astype(np.float32)
        X[rng.random((S, F)) < 0.3] = np.nan
        rp, pp, n_p = orc.pearson(X)
        rs, ps, n_s = orc.spearman(X)
        for g, h in itertools.product(range(F), repeat=2):
            keep = [i for i in range(S) if not (np.isnan(X[i, g]) or np.isnan(X[i, h]))]
            assert n_p[g, h] == len(keep) == n_s[g, h]
            a = [X[i, g] for i in keep]
            b = [X[i, h] for i in keep]
            if len(keep) <= 1:
                assert math.isnan(rp[g, h]) and math.isnan(rs[g, h])
                continue
            r2, sgn = _exact_r2_and_sign(a, b)
            if r2 is None:
                assert math.isnan(rp[g, h])
            else:
                assert abs(rp[g, h] ** 2 - float(r2)) <= 1e-13
                if float(r2) > 1e-20:
                    assert np.sign(rp[g, h]) == sgn
            ra, rb = _exact_avg_ranks(a), _exact_avg_ranks(b)
            r2s, sgns = _exact_r2_and_sign([float(x) for x in ra], [float(x) for x in rb])
            if r2s is None:
                assert math.isnan(rs[g, h])
            else:
                assert abs(rs[g, h] ** 2 - float(r2s)) <= 1e-13
                if float(r2s) > 1e-20:
                    assert np.sign(rs[g, h]) == sgns


def test_pair_ranks_match_counting_definition():
    X = synth.heavy_ties(60, 4, levels=4, missing=0.25, seed=5)
    for g, h in [(0, 1), (2, 3), (1, 1)]:
        rg, rh, n = orc.pair_ranks(X, g, h)
        keep = ~(np.isnan(X[:, g]) | np.isnan(X[:, h]))
        assert n == keep.sum()
        assert np.all(np.isnan(rg[~keep])) and np.all(np.isnan(rh[~keep]))
        ref_g = _exact_avg_ranks(list(X[keep, g]))
        ref_h = _exact_avg_ranks(list(X[keep, h]))
        assert np.array_equal(rg[keep], np.array([float(x) for x in ref_g]))
        assert np.array_equal(rh[keep], np.array([float(x) for x in ref_h]))
        # doubled ranks are integers summing to n(n+1)
        assert np.all((2 * rg[keep]) == np.round(2 * rg[keep]))
        assert (2 * rg[keep]).sum() == n * (n + 1)


# --------------------------------------------------------------------------
# library routines
# --------------------------------------------------------------------------

def test_no_missing_matches_numpy_corrcoef():
    rng = np.random.default_rng(3)
    X = (rng.standard_normal((200, 12)) @ rng.standard_normal((12, 12))).astype(np.float32)
    r, p, n = orc.pearson(X)
    ref = np.corrcoef(X.astype(np.float64), rowvar=False)
    assert np.max(np.abs(r - ref)) <= 1e-12
    assert np.all(n == 200)


def test_pairwise_deletion_matches_pandas():
    pd = pytest.importorskip("pandas")
    X = synth.cfg_plain_small()
    df = pd.DataFrame(X.astype(np.float64))
    r, _, _ = orc.pearson(X)
    ref = df.corr(method="pearson").to_numpy()
    both = np.isfinite(ref) & np.isfinite(r)
    assert np.array_equal(np.isfinite(ref), np.isfinite(r))
    assert np.max(np.abs(r[both] - ref[both])) <= 1e-12
    rs, _, _ = orc.spearman(X)
    ref_s = df.corr(method="spearman").to_numpy()
    assert np.max(np.abs(rs - ref_s)) <= 1e-12


def test_spearman_matches_scipy_omit_and_pvalues():
    from scipy import stats
    X = synth.cfg_plain_small()
    rs, ps, ns = orc.spearman(X)
    rp, pp, npp = orc.pearson(X)
    for g, h in [(0, 1), (3, 17), (10, 42), (49, 2), (5, 5)]:
        x, y = X[:, g].astype(np.float64), X[:, h].astype(np.float64)
        keep = ~(np.isnan(x) | np.isnan(y))
        res = stats.spearmanr(x, y, nan_policy="omit")
        assert abs(rs[g, h] - res.statistic) <= 1e-12
        if g != h:
            assert abs(ps[g, h] - res.pvalue) <= 1e-12 * max(1.0, abs(res.pvalue))
        pr = stats.pearsonr(x[keep], y[keep])
        assert abs(rp[g, h] - pr.statistic) <= 1e-12
        if g != h:
            assert abs(pp[g, h] - pr.pvalue) <= 1e-10 * max(pr.pvalue, 1e-300)


def test_spearman_no_ties_closed_form():
    """Without ties and missing values rho = 1 - 6 sum d^2 / (n (n^2 - 1))."""
    rng = np.random.default_rng(8)
    X = rng.standard_normal((97, 6)).astype(np.float32)
    X[:, 3] = X[:, 0] + 0.3 * X[:, 3]
    rs, _, _ = orc.spearman(X)
    n = X.shape[0]
    ranks = np.argsort(np.argsort(X, axis=0), axis=0) + 1
    for g, h in itertools.combinations(range(6), 2):
        d = (ranks[:, g] - ranks[:, h]).astype(np.int64)
        ref = 1.0 - 6.0 * float((d * d).sum()) / (n * (n * n - 1))
        assert abs(rs[g, h] - ref) <= 1e-13


# --------------------------------------------------------------------------
# the p-value function
# --------------------------------------------------------------------------

@pytest.mark.parametrize("r", [0.0, 0.1, -0.37, 0.5, 0.9, -0.999])
def test_pvalue_closed_forms_small_n(r):
    # n = 3: p = 1 - (2/pi) asin|r| ; n = 4: p = 1 - |r|
    p3 = orc.pvalue(np.array([r]), np.array([3]), "pearson")[0]
    p4 = orc.pvalue(np.array([r]), np.array([4]), "spearman")[0]
    assert abs(p3 - (1 - 2 / math.pi * math.asin(abs(r)))) <= 1e-14
    assert abs(p4 - (1 - abs(r))) <= 1e-14


def test_pvalue_against_mpmath():
    rng = np.random.default_rng(4)
    for _ in range(40):
        n = int(rng.choice([5, 10, 37, 100, 1000, 6650, 20000]))
        r = float(rng.uniform(-0.3, 0.3)) if n > 1000 else float(rng.uniform(-0.99, 0.99))
        p = orc.pvalue(np.array([r]), np.array([n]), "pearson")[0]
        ref = orc.pvalue_mp(r, n)
        assert abs(p - ref) <= 1e-12 * max(ref, 1e-300), (n, r, p, ref)


@pytest.mark.parametrize("r", [1e-12, -3e-9, 2e-8, 1e-6])
def test_pvalue_tiny_r(r):
    """1 - r^2 rounds to 1 in FP64 for these r; p must still fall below 1 by
    the right amount.  n = 3, 4: the closed forms; large n: the leading term
    of I_y(1/2, a) as y -> 0, which is 2 sqrt(y) / B(1/2, a), so
    1 - p = 2|r| / B(1/2, a) up to a relative O(a r^2) correction."""
    p3 = orc.pvalue(np.array([r]), np.array([3]), "pearson")[0]
    p4 = orc.pvalue(np.array([r]), np.array([4]), "pearson")[0]
    assert abs((1 - p3) - 2 / math.pi * math.asin(abs(r))) <= 1e-15
    assert abs((1 - p4) - abs(r)) <= 1e-15
    for n in (1000, 28000):
        a = (n - 2) / 2
        lnB = math.lgamma(0.5) + math.lgamma(a) - math.lgamma(a + 0.5)
        q = 2 * abs(r) / math.exp(lnB)
        p = orc.pvalue(np.array([r]), np.array([n]), "pearson")[0]
        assert abs((1 - p) - q) <= 2e-15 + 1e-6 * q, (n, r, 1 - p, q)
        assert abs(p - orc.pvalue_mp(r, n)) <= 1e-15


def test_pvalue_equals_student_t_tail():
    from scipy import stats
    for n in (3, 4, 5, 10, 1000):
        for r in (0.05, 0.3, -0.7):
            df = n - 2
            t = r * math.sqrt(df / (1 - r * r))
            ref = 2 * stats.t.sf(abs(t), df)
            p = orc.pvalue(np.array([r]), np.array([n]), "spearman")[0]
            assert abs(p - ref) <= 1e-12 * ref


def test_pvalue_undefined_cases():
    r = np.array([0.5, 0.5, 0.5, np.nan, 1.0])
    n = np.array([1, 2, 2, 10, 5])
    pp = orc.pvalue(r, n, "pearson")
    ps = orc.pvalue(r, n, "spearman")
    assert math.isnan(pp[0]) and pp[1] == 1.0 and pp[2] == 1.0 and math.isnan(pp[3]) and pp[4] == 0.0
    assert math.isnan(ps[0]) and math.isnan(ps[1]) and math.isnan(ps[3]) and ps[4] == 0.0


# --------------------------------------------------------------------------
# invariants
# --------------------------------------------------------------------------

def test_invariants():
    X = synth.cfg_plain_small(F=20)
    rng = np.random.default_rng(9)
    rp, _, n = orc.pearson(X)
    rs, _, _ = orc.spearman(X)
    for r in (rp, rs):
        assert np.array_equal(r, r.T, equal_nan=True)
        assert np.nanmax(np.abs(r)) <= 1.0
        assert np.allclose(np.diag(r), 1.0, atol=1e-15)
    assert np.array_equal(n, n.T)
    # row permutation: counts exact, r to rounding
    perm = rng.permutation(X.shape[0])
    rp2, _, n2 = orc.pearson(X[perm])
    rs2, _, _ = orc.spearman(X[perm])
    assert np.array_equal(n, n2)
    assert np.max(np.abs(rp - rp2)) <= 1e-12
    assert np.max(np.abs(rs - rs2)) <= 1e-12
    # column permutation: equivariance
    cp = rng.permutation(X.shape[1])
    rp3, _, n3 = orc.pearson(X[:, cp])
    assert np.array_equal(n3, n[np.ix_(cp, cp)])
    assert np.max(np.abs(rp3 - rp[np.ix_(cp, cp)])) <= 1e-12
    # positive affine map of a column leaves Pearson unchanged; negative flips it
    Xa = X.astype(np.float64).copy()
    Xa[:, 4] = 2.0 * Xa[:, 4] + 5.0
    Xa[:, 7] = -0.5 * Xa[:, 7] + 1.0
    rpa, _, _ = orc.pearson(Xa)
    mask = np.arange(20) != 7
    assert np.max(np.abs(rpa[4][mask] - rp[4][mask])) <= 1e-12
    assert abs(rpa[4, 7] + rp[4, 7]) <= 1e-12
    mask &= np.arange(20) != 4
    assert np.max(np.abs(rpa[7][mask] + rp[7][mask])) <= 1e-12
    # strictly increasing transform leaves Spearman unchanged exactly
    Xm = X.astype(np.float64).copy()
    Xm[:, 2] = np.exp(Xm[:, 2] / 3.0)
    Xm[:, 5] = Xm[:, 5] ** 3
    rsm, _, _ = orc.spearman(Xm)
    assert np.max(np.abs(rsm - rs)) <= 1e-13


def test_exact_linear_and_monotone_relations():
    rng = np.random.default_rng(2)
    x = rng.standard_normal(300)
    X = np.stack([x, 3 * x - 1, -0.25 * x + 7, np.exp(x), -(x ** 3)], axis=1)
    X[rng.random(X.shape) < 0.2] = np.nan
    rp, _, _ = orc.pearson(X)
    rs, _, _ = orc.spearman(X)
    assert abs(rp[0, 1] - 1) <= 1e-12 and abs(rp[0, 2] + 1) <= 1e-12
    assert rs[0, 3] == 1.0 and rs[0, 4] == -1.0 and rs[3, 4] == -1.0


def test_sentinel_missing_value():
    X = synth.cfg_plain_small(F=8).astype(np.float64)
    Xs = np.where(np.isnan(X), -999.0, X)
    r1, p1, n1 = orc.pearson(X)
    r2, p2, n2 = orc.pearson(Xs, missing=-999.0)
    assert np.array_equal(n1, n2)
    assert np.array_equal(r1, r2, equal_nan=True)


# --------------------------------------------------------------------------
# the reference gradient
# --------------------------------------------------------------------------

def test_reference_gradient_finite_differences():
    case = synth.cfg_differentiation(S=64, F=6, n_fd=12)
    X = case.X.astype(np.float64)
    W = case.W[:6, :6]
    loss, g, r = ograd.pearson_loss_grad(X, W)
    # the autograd forward is the oracle's Pearson
    ro, _, no = orc.pearson(X)
    off = ~np.eye(6, dtype=bool)
    assert np.max(np.abs(r[off] - ro[off])) <= 1e-12
    assert abs(loss - ograd.pearson_loss(X, W)) <= 1e-12
    h = 1e-5
    for (i, c) in case.fd_entries:
        Xp = X.copy()
        Xm = X.copy()
        Xp[i, c] += h
        Xm[i, c] -= h
        fd = (ograd.pearson_loss(Xp, W) - ograd.pearson_loss(Xm, W)) / (2 * h)
        assert abs(fd - g[i, c]) <= 1e-6 * max(1.0, abs(fd)), (i, c, fd, g[i, c])
    for (i, c) in case.nan_entries:
        assert g[i, c] == 0.0
