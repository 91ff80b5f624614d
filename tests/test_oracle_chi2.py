"""Pins of the chi-squared oracle (oracle/chi2.py), CPU only: SciPy's
chi2_contingency without continuity correction, the 2 x 2 closed form,
an exactly independent table, symmetry, label relabelling and the paper's
undefined cases."""

import numpy as np
import pytest
from scipy import stats

from oracle import chi2 as oc


@pytest.mark.parametrize("shape", [(2, 2), (2, 5), (4, 3), (7, 7)])
def test_table_matches_scipy(shape):
    rng = np.random.default_rng(shape[0] * 10 + shape[1])
    O = rng.integers(1, 40, size=shape).astype(float)
    chi2, p, V = oc.table_test(O)
    ref = stats.chi2_contingency(O, correction=False)
    np.testing.assert_allclose(chi2, ref.statistic, rtol=1e-12)
    np.testing.assert_allclose(p, ref.pvalue, rtol=1e-10)
    np.testing.assert_allclose(V, stats.contingency.association(O.astype(int), method="cramer"), rtol=1e-12)


def test_closed_forms():
    a, b, c, d = 12.0, 5.0, 7.0, 19.0
    N = a + b + c + d
    chi2, p, V = oc.table_test(np.array([[a, b], [c, d]]))
    ref = N * (a * d - b * c) ** 2 / ((a + b) * (c + d) * (a + c) * (b + d))
    np.testing.assert_allclose(chi2, ref, rtol=1e-13)
    np.testing.assert_allclose(V, np.sqrt(ref / N), rtol=1e-13)  # phi
    # exactly independent table: O = E
    chi2, p, V = oc.table_test(np.outer([2.0, 3.0, 5.0], [4.0, 6.0]))
    assert abs(chi2) < 1e-12 and abs(p - 1.0) < 1e-12


def test_undefined_cases():
    # a category empty: everything NaN
    assert all(np.isnan(v) for v in oc.table_test(np.array([[3.0, 0.0], [4.0, 0.0]])))
    # a single category on one side: chi2 = 0, p and V NaN
    chi2, p, V = oc.table_test(np.array([[3.0, 4.0, 5.0]]))
    assert chi2 == 0.0 and np.isnan(p) and np.isnan(V)


def test_matrix_symmetry_relabelling_and_deletion():
    rng = np.random.default_rng(4)
    S = 200
    L = np.column_stack([rng.integers(0, 3, S), rng.integers(0, 2, S), rng.integers(0, 4, S)]).astype(np.float32)
    L[:, 2] = np.where(rng.random(S) < 0.5, L[:, 0], L[:, 2])  # dependence
    L[rng.random((S, 3)) < 0.15] = np.nan
    c2, p, V, n = oc.chi2(L)
    np.testing.assert_allclose(c2, c2.T, rtol=1e-14)  # transposed table: summation order only
    np.testing.assert_array_equal(n, n.T)
    # relabelling the categories of a feature changes nothing
    L2 = L.copy()
    L2[:, 0] = np.where(np.isnan(L[:, 0]), np.nan, 2.0 - L[:, 0])
    c2b, pb, Vb, nb = oc.chi2(L2)
    np.testing.assert_allclose(c2b, c2, rtol=1e-12)
    # pairwise deletion by hand for (0, 2)
    keep = ~np.isnan(L[:, 0]) & ~np.isnan(L[:, 2])
    O = np.array([[np.sum((L[keep, 0] == u) & (L[keep, 2] == v)) for v in range(4)] for u in range(3)], float)
    ref = stats.chi2_contingency(O, correction=False)
    np.testing.assert_allclose([c2[0, 2], p[0, 2]], [ref.statistic, ref.pvalue], rtol=1e-10)
    assert n[0, 2] == keep.sum()
    # a label at the caller's bound: the column is not tested
    c3, _, _, n3 = oc.chi2(L, ncat=3)
    assert np.all(np.isnan(c3[2])) and np.all(n3[2] == 0) and not np.isnan(c3[0, 1])
