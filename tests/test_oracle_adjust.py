"""Pins of the multiple-testing oracle (oracle/adjust.py), CPU only.

The definitions are checked against SciPy's false_discovery_control (BH and
BY), against the minimum over l >= k written out in loops on tiny inputs,
against closed forms and against invariants that a dropped term, a wrong rank
or a double-counted test would break.
"""

import math

import numpy as np
import pytest
from scipy.stats import false_discovery_control

from oracle import adjust


def _pvals(rng, m, ties=True):
    p = rng.random(m) ** 3
    if ties and m > 4:
        p[:: 5] = p[1]  # groups of equal p-values
        p[2] = 0.0
        p[3] = 1.0
    return p


@pytest.mark.parametrize("method", ["bh", "by"])
@pytest.mark.parametrize("m", [1, 2, 7, 100, 5000])
def test_matches_scipy(method, m):
    rng = np.random.default_rng(2505 + m)
    p = _pvals(rng, m)
    got = adjust.adjust_vector(p, method)
    ref = false_discovery_control(p, method=method)
    np.testing.assert_allclose(got, ref, rtol=1e-14, atol=0)


@pytest.mark.parametrize("method", ["bonferroni", "bh", "by"])
def test_brute_force_tiny(method):
    rng = np.random.default_rng(7)
    for m in range(1, 10):
        for _ in range(20):
            p = np.round(rng.random(m), 1)  # many ties
            got = adjust.adjust_vector(p, method)
            ref = adjust.adjust_brute(p, method)
            np.testing.assert_allclose(got, ref, rtol=1e-15, atol=0)


def test_closed_forms():
    # one test: nothing to adjust
    for method in adjust.METHODS:
        assert adjust.adjust_vector(np.array([0.03]), method)[0] == 0.03
    # m equal p-values: BH leaves them unchanged, BY multiplies by c(m)
    p = np.full(6, 0.01)
    np.testing.assert_allclose(adjust.adjust_vector(p, "bh"), p, rtol=1e-15)
    c6 = 1 + 1 / 2 + 1 / 3 + 1 / 4 + 1 / 5 + 1 / 6
    np.testing.assert_allclose(adjust.adjust_vector(p, "by"), p * c6, rtol=1e-15)
    np.testing.assert_allclose(adjust.adjust_vector(p, "bonferroni"), 6 * p, rtol=1e-15)
    # BH step-up on a hand-worked set of four: p = .01, .02, .03, .5 ->
    # m p / k = .04, .04, .04, .5
    np.testing.assert_allclose(adjust.adjust_vector(np.array([0.03, 0.01, 0.5, 0.02]), "bh"),
                               [0.04, 0.04, 0.5, 0.04], rtol=1e-15)
    assert math.isclose(adjust.harmonic(4), 25 / 12, rel_tol=1e-16)


@pytest.mark.parametrize("m", [3, 50, 3000])
def test_invariants(m):
    rng = np.random.default_rng(m)
    p = _pvals(rng, m)
    bon = adjust.adjust_vector(p, "bonferroni")
    bh = adjust.adjust_vector(p, "bh")
    by = adjust.adjust_vector(p, "by")
    for a in (bon, bh, by):
        assert np.all(a >= p) and np.all(a <= 1.0)
        # order preserving: a smaller p never gets a larger adjusted value
        o = np.argsort(p, kind="stable")
        assert np.all(np.diff(a[o]) >= 0)
        # equal p-values get equal adjusted values
        assert np.all(a[p == p[1]] == a[1])
    assert np.all(by >= bh) and np.all(bon >= bh)
    # permutation invariance
    perm = rng.permutation(m)
    np.testing.assert_array_equal(adjust.adjust_vector(p[perm], "bh"), bh[perm])


def test_matrix_counts_each_pair_once_and_skips_nan():
    F = 5
    P = np.full((F, F), 1e-6)
    out = adjust.adjust_matrix(P, "bonferroni")
    assert np.all(np.isnan(np.diag(out)))
    off = out[~np.eye(F, dtype=bool)]
    np.testing.assert_allclose(off, 10e-6, rtol=1e-15)  # F (F - 1) / 2 = 10 tests
    # an undefined pair is not a test: 9 tests remain
    P[1, 3] = P[3, 1] = np.nan
    out = adjust.adjust_matrix(P, "bonferroni")
    assert np.isnan(out[1, 3]) and np.isnan(out[3, 1])
    np.testing.assert_allclose(out[0, 1], 9e-6, rtol=1e-15)
    # the result is symmetric and read from the upper triangle
    rng = np.random.default_rng(3)
    A = rng.random((F, F))
    S = np.triu(A, 1) + np.triu(A, 1).T
    for method in adjust.METHODS:
        o = adjust.adjust_matrix(S, method)
        np.testing.assert_array_equal(o, o.T)
        iu = np.triu_indices(F, 1)
        np.testing.assert_allclose(o[iu], adjust.adjust_vector(S[iu], method), rtol=0)
