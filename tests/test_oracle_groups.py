"""Pins of the t-test / ANOVA oracle (oracle/groups.py), CPU only.

Checked against SciPy's ttest_ind (Student and Welch) and f_oneway on
per-pair data drawn independently of the oracle's deletion code, against the
identity F = t^2 (and equal p) of a two-group ANOVA and Student's t, against
invariances (shift, scale, label swap), hand-built pairwise deletion and the
paper's undefined cases.
"""

import numpy as np
import pytest
from scipy import stats

from oracle import groups as og


def _pair_data(rng, n0, n1, mu=(0.0, 0.7), sd=(1.0, 2.0)):
    y0 = rng.normal(mu[0], sd[0], n0)
    y1 = rng.normal(mu[1], sd[1], n1)
    return y0, y1


@pytest.mark.parametrize("welch", [False, True])
@pytest.mark.parametrize("n0,n1", [(2, 2), (2, 9), (30, 17), (400, 1200)])
def test_ttest_matches_scipy(welch, n0, n1):
    rng = np.random.default_rng(n0 * 1000 + n1)
    y0, y1 = _pair_data(rng, n0, n1)
    t, p = og.ttest_pair(y0, y1, welch)
    ref = stats.ttest_ind(y0, y1, equal_var=not welch)
    np.testing.assert_allclose(t, ref.statistic, rtol=1e-12)
    np.testing.assert_allclose(p, ref.pvalue, rtol=1e-10)


@pytest.mark.parametrize("K", [2, 3, 5])
def test_anova_matches_scipy_and_two_group_identity(K):
    rng = np.random.default_rng(K)
    groups = [rng.normal(0.3 * k, 1.0 + 0.2 * k, 5 + 7 * k) for k in range(K)]
    F, p = og.anova_groups(groups)
    ref = stats.f_oneway(*groups)
    np.testing.assert_allclose(F, ref.statistic, rtol=1e-12)
    np.testing.assert_allclose(p, ref.pvalue, rtol=1e-10)
    if K == 2:
        t, pt = og.ttest_pair(groups[0], groups[1], welch=False)
        np.testing.assert_allclose(F, t * t, rtol=1e-12)
        np.testing.assert_allclose(p, pt, rtol=1e-10)


def test_invariances():
    rng = np.random.default_rng(5)
    y0, y1 = _pair_data(rng, 40, 55)
    for welch in (False, True):
        t, p = og.ttest_pair(y0, y1, welch)
        t2, p2 = og.ttest_pair(3.0 * y0 + 1e4, 3.0 * y1 + 1e4, welch)  # affine change of x
        np.testing.assert_allclose([t2, p2], [t, p], rtol=1e-9)
        t3, p3 = og.ttest_pair(y1, y0, welch)  # labels swapped
        np.testing.assert_allclose([t3, p3], [-t, p], rtol=1e-14)
    gs = [y0, y1, rng.normal(0, 1, 30)]
    F, p = og.anova_groups(gs)
    F2, p2 = og.anova_groups([2.5 * g - 7.0 for g in gs])
    np.testing.assert_allclose([F2, p2], [F, p], rtol=1e-9)


def test_undefined_cases():
    a = np.array([1.0, 2.0, 3.0])
    # a group with fewer than two samples
    assert np.isnan(og.ttest_pair(a, np.array([5.0]), False)[0])
    assert np.isnan(og.ttest_pair(np.array([5.0]), a, True)[0])
    # zero pooled standard deviation: Student NaN; Welch +-inf / NaN
    c0, c1 = np.array([2.0, 2.0, 2.0]), np.array([4.0, 4.0])
    assert np.isnan(og.ttest_pair(c0, c1, False)[0])
    assert og.ttest_pair(c0, c1, True) == (-np.inf, 0.0)
    assert np.isnan(og.ttest_pair(c0, c0[:2], True)[0])
    # ANOVA: empty category, single category, zero within-category variance
    assert np.isnan(og.anova_groups([a, np.array([])])[0])
    assert np.isnan(og.anova_groups([a])[0])
    assert og.anova_groups([c0, c1, np.array([9.0])]) == (np.inf, 0.0)
    assert np.isnan(og.anova_groups([c0, c0[:1]])[0])


def test_matrix_pairwise_deletion_by_hand():
    """The matrix driver against per-pair inputs assembled by hand."""
    rng = np.random.default_rng(11)
    S = 60
    L = rng.integers(0, 3, size=(S, 2)).astype(np.float32)
    L[:, 1] = rng.integers(0, 2, size=S)
    X = rng.normal(size=(S, 3)).astype(np.float32)
    L[rng.random((S, 2)) < 0.2] = np.nan
    X[rng.random((S, 3)) < 0.2] = np.nan
    F, pF, n = og.anova(L, X)
    t, pt, nt = og.ttest(L, X, welch=True)
    for j in range(3):
        keep = ~np.isnan(L[:, 0]) & ~np.isnan(X[:, j])
        gs = [X[keep & (L[:, 0] == k), j].astype(np.float64) for k in range(3)]
        ref = stats.f_oneway(*gs)
        np.testing.assert_allclose([F[0, j], pF[0, j]], [ref.statistic, ref.pvalue], rtol=1e-10)
        assert n[0, j] == keep.sum()
        keep = ~np.isnan(L[:, 1]) & ~np.isnan(X[:, j])
        y0 = X[keep & (L[:, 1] == 0), j].astype(np.float64)
        y1 = X[keep & (L[:, 1] == 1), j].astype(np.float64)
        ref = stats.ttest_ind(y0, y1, equal_var=False)
        np.testing.assert_allclose([t[1, j], pt[1, j]], [ref.statistic, ref.pvalue], rtol=1e-10)
        assert nt[1, j] == keep.sum()
    # column 0 has three labels: not dichotomous, so its t-tests are NaN, n 0
    assert np.all(np.isnan(t[0])) and np.all(nt[0] == 0)
    # a category bound below the largest label: column 0 not tested
    F2, _, n2 = og.anova(L, X, ncat=2)
    assert np.all(np.isnan(F2[0])) and np.all(n2[0] == 0)
    np.testing.assert_array_equal(F2[1], F[1])


def test_sentinel_and_listed_pairs():
    rng = np.random.default_rng(3)
    L = rng.integers(0, 2, size=(50, 3)).astype(np.float32)
    X = rng.normal(size=(50, 4)).astype(np.float32)
    Ls, Xs = L.copy(), X.copy()
    L[5, 1] = np.nan
    Ls[5, 1] = -9.0
    X[7, 2] = np.nan
    Xs[7, 2] = -9.0
    a = og.ttest(L, X)
    b = og.ttest(Ls, Xs, missing=-9.0)
    for u, v in zip(a, b):
        np.testing.assert_array_equal(u, v)
    pairs = [(2, 3), (0, 0), (1, 2)]
    s, p, n = og.ttest(L, X, pairs=pairs)
    for k, (i, j) in enumerate(pairs):
        assert (s[k], p[k], n[k]) == (a[0][i, j], a[1][i, j], a[2][i, j])
