"""Pins of the Mann-Whitney / Kruskal-Wallis oracle (oracle/ranktests.py),
CPU only: SciPy's mannwhitneyu (with the method the paper's rule picks) and
kruskal, brute-force enumeration of the exact U distribution, the two-group
identity H = z^2 (no ties, no continuity correction), invariances and the
undefined cases."""

import itertools
import math

import numpy as np
import pytest
from scipy import stats

from oracle import ranktests as orank


@pytest.mark.parametrize("n0,n1,ties", [(3, 5, False), (7, 40, False), (8, 8, False), (30, 45, True),
                                        (500, 700, True), (2, 3, True)])
def test_mwu_matches_scipy(n0, n1, ties):
    rng = np.random.default_rng(n0 * 100 + n1)
    y0 = rng.normal(0.0, 1.0, n0)
    y1 = rng.normal(0.4, 1.0, n1)
    if ties:
        y0, y1 = np.round(y0, 1), np.round(y1, 1)
    U, p = orank.mwu_pair(y0, y1)
    has_ties = np.unique(np.concatenate([y0, y1])).size < n0 + n1
    method = "exact" if (not has_ties and min(n0, n1) < 8) else "asymptotic"
    ref = stats.mannwhitneyu(y0, y1, method=method)
    np.testing.assert_allclose(U, ref.statistic, rtol=1e-14)
    np.testing.assert_allclose(p, ref.pvalue, rtol=1e-10)


def test_exact_distribution_brute_force():
    for m, M in [(1, 1), (1, 4), (2, 3), (3, 3), (4, 5), (3, 7)]:
        N = m + M
        counts = {}
        for pos in itertools.combinations(range(1, N + 1), m):
            u = sum(pos) - m * (m + 1) // 2
            counts[u] = counts.get(u, 0) + 1
        total = math.comb(N, m)
        for u in range(0, m * M + 2):
            ref = sum(c for k, c in counts.items() if k >= u) / total
            assert abs(orank.mwu_exact_sf(u, m, M) - ref) < 1e-14
            assert abs(orank.mwu_exact_sf(u, M, m) - ref) < 1e-14  # symmetric in the sizes


@pytest.mark.parametrize("K,ties", [(2, False), (3, True), (5, False), (6, True)])
def test_kruskal_matches_scipy(K, ties):
    rng = np.random.default_rng(K + 10 * ties)
    groups = [rng.normal(0.2 * k, 1.0, 6 + 5 * k) for k in range(K)]
    if ties:
        groups = [np.round(g, 1) for g in groups]
    H, p = orank.kruskal_groups(groups)
    ref = stats.kruskal(*groups)
    np.testing.assert_allclose(H, ref.statistic, rtol=1e-12)
    np.testing.assert_allclose(p, ref.pvalue, rtol=1e-10)


def test_two_group_identity_and_invariances():
    rng = np.random.default_rng(2)
    y0, y1 = rng.normal(0, 1, 25), rng.normal(0.5, 1, 31)
    H, _ = orank.kruskal_groups([y0, y1])
    U, _ = orank.mwu_pair(y0, y1)
    n0, n1 = y0.size, y1.size
    z2 = (U - n0 * n1 / 2) ** 2 / (n0 * n1 * (n0 + n1 + 1) / 12)
    np.testing.assert_allclose(H, z2, rtol=1e-12)
    # a monotone transform of the values changes nothing
    U2, p2 = orank.mwu_pair(np.exp(y0), np.exp(y1))
    assert U2 == U
    # swapping the groups: U1 -> n0 n1 - U1, same p
    Us, ps = orank.mwu_pair(y1, y0)
    _, p = orank.mwu_pair(y0, y1)
    assert Us == n0 * n1 - U and ps == p


def test_undefined_cases():
    a = np.array([1.0, 2.0, 3.0])
    assert np.isnan(orank.mwu_pair(a, np.array([]))[0])
    # all values tied: MWU p = 1, Kruskal-Wallis undefined
    c = np.array([2.0, 2.0, 2.0])
    U, p = orank.mwu_pair(c, c[:2])
    assert U == 3.0 and p == 1.0
    assert np.isnan(orank.kruskal_groups([c, c[:2]])[0])
    assert np.isnan(orank.kruskal_groups([a])[0])
    assert np.isnan(orank.kruskal_groups([a, np.array([])])[0])


def test_matrix_pairwise_deletion_by_hand():
    rng = np.random.default_rng(12)
    S = 80
    L = np.column_stack([rng.integers(0, 2, S), rng.integers(0, 3, S)]).astype(np.float32)
    X = np.round(rng.normal(size=(S, 3)), 1).astype(np.float32)
    L[rng.random((S, 2)) < 0.2] = np.nan
    X[rng.random((S, 3)) < 0.2] = np.nan
    U, pU, nU = orank.mannwhitney(L, X)
    H, pH, nH = orank.kruskal(L, X)
    for j in range(3):
        keep = ~np.isnan(L[:, 0]) & ~np.isnan(X[:, j])
        y0 = X[keep & (L[:, 0] == 0), j].astype(np.float64)
        y1 = X[keep & (L[:, 0] == 1), j].astype(np.float64)
        ref = stats.mannwhitneyu(y0, y1, method="asymptotic")  # ties present
        np.testing.assert_allclose([U[0, j], pU[0, j]], [ref.statistic, ref.pvalue], rtol=1e-10)
        assert nU[0, j] == keep.sum()
        keep = ~np.isnan(L[:, 1]) & ~np.isnan(X[:, j])
        ref = stats.kruskal(*[X[keep & (L[:, 1] == k), j].astype(np.float64) for k in range(3)])
        np.testing.assert_allclose([H[1, j], pH[1, j]], [ref.statistic, ref.pvalue], rtol=1e-10)
    assert np.all(np.isnan(U[1])) and np.all(nU[1] == 0)  # three labels: not dichotomous
