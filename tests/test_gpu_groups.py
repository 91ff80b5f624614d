"""GPU parity of the categorical x continuous tests (napy_ttest, napy_anova)
against the FP64 oracle (oracle/groups.py) on seeded synthetic inputs.

Both sides work in FP64; the device sums run through FP64 matrix cores in a
different order and about the column mean, so statistics agree to a relative
1e-9 (plus 1e-12 absolute for statistics near zero).  The oracle's p-values
come from SciPy's t and F tails, which are accurate to about 1e-9 relative at
these degrees of freedom; the device's own tail is pinned to 1e-10 against a
40-digit reference in test_abi.py.  So p agrees to 1e-8 relative.
Undefined results (NaN), infinities and the counts n must match exactly.
"""

import numpy as np
import pytest

from oracle import groups as og

pytestmark = pytest.mark.gpu


def _check(got, ref, what):
    s, p, n = got
    rs, rp, rn = ref
    assert np.array_equal(np.isnan(s), np.isnan(rs)), f"{what}: NaN placement of the statistic differs"
    assert np.array_equal(np.isnan(p), np.isnan(rp)), f"{what}: NaN placement of p differs"
    assert np.array_equal(np.isinf(s), np.isinf(rs)), f"{what}: infinities differ"
    fin = np.isfinite(rs)
    assert np.all(np.sign(s[np.isinf(rs)]) == np.sign(rs[np.isinf(rs)]))
    np.testing.assert_allclose(s[fin], rs[fin], rtol=1e-9, atol=1e-12, err_msg=what)
    ok = ~np.isnan(rp)
    np.testing.assert_allclose(p[ok], rp[ok], rtol=1e-8, atol=1e-300, err_msg=what)
    np.testing.assert_array_equal(n, rn, err_msg=what)


def _with_edges(L, X, ncat):
    """Append degenerate columns: a dichotomous column with one group, one with
    an out-of-range label, one with a non-integer label, an all-missing one;
    continuous columns constant overall, constant within the groups of
    categorical column 0 (different means), and all missing."""
    S = L.shape[0]
    rng = np.random.default_rng(99)
    one_group = np.zeros(S)
    out_of_range = L[:, 0].copy()
    out_of_range[3] = ncat
    non_int = L[:, 0].copy()
    non_int[4] = 0.5
    all_missing = np.full(S, np.nan)
    L2 = np.column_stack([L, one_group, out_of_range, non_int, all_missing]).astype(np.float32)
    const = np.full(S, 3.25)
    const[rng.random(S) < 0.2] = np.nan
    by_group = np.where(np.isnan(L[:, 0]), np.nan, 2.0 * np.nan_to_num(L[:, 0]) + 1.0)
    X2 = np.column_stack([X, const, by_group, np.full(S, np.nan)]).astype(np.float32)
    return L2, X2


def _run_gpu(kind, L, X, gpu_device, **kw):
    import torch
    import paper_2505_00448_amd as napy
    Lt = torch.from_numpy(L).to(gpu_device)
    Xt = torch.from_numpy(X).to(gpu_device)
    if kind == "ttest":
        out = napy.ttest(Lt, Xt, **kw)
        return out["t"].cpu().numpy(), out["p"].cpu().numpy(), out["n"].cpu().numpy()
    out = napy.anova(Lt, Xt, **kw)
    return out["F"].cpu().numpy(), out["p"].cpu().numpy(), out["n"].cpu().numpy()


@pytest.mark.parametrize("welch", [False, True])
def test_ttest_matches_oracle(gpu_device, welch):
    import synth
    print(f"ttest welch={welch}", flush=True)
    L, X = synth.categorical_continuous(777, 13, 130, 2, seed=5)
    L, X = _with_edges(L, X, 2)
    got = _run_gpu("ttest", L, X, gpu_device, welch=welch)
    ref = og.ttest(L, X, welch=welch)
    _check(got, ref, f"ttest welch={welch}")
    # the edge columns behave as the paper says
    s = got[0]
    FC = L.shape[1]
    assert np.all(np.isnan(s[FC - 4])) and np.all(np.isnan(s[FC - 3])) and np.all(np.isnan(s[FC - 2]))
    assert np.all(got[2][FC - 3] == 0)


@pytest.mark.parametrize("ncat", [3, 4, 9])
def test_anova_matches_oracle(gpu_device, ncat):
    import synth
    print(f"anova ncat={ncat}", flush=True)
    L, X = synth.categorical_continuous(1500, 20, 70, ncat, seed=ncat)
    L, X = _with_edges(L, X, ncat)
    got = _run_gpu("anova", L, X, gpu_device, ncat=ncat)
    ref = og.anova(L, X, ncat=ncat)
    _check(got, ref, f"anova ncat={ncat}")
    # categorical column 0 against the column constant within its groups
    FQ = X.shape[1]
    assert got[0][0, FQ - 2] == np.inf and got[1][0, FQ - 2] == 0.0


def test_anova_empty_category_within_pair(gpu_device):
    """A category observed in the column but only where x is missing: the
    pair's test is undefined while other pairs of the column are not."""
    print("anova empty category", flush=True)
    rng = np.random.default_rng(8)
    S = 300
    L = rng.integers(0, 3, size=(S, 2)).astype(np.float32)
    X = rng.normal(size=(S, 3)).astype(np.float32)
    X[L[:, 0] == 2, 1] = np.nan  # category 2 of column 0 empty for pair (0, 1)
    got = _run_gpu("anova", L, X, gpu_device, ncat=3)
    ref = og.anova(L, X, ncat=3)
    _check(got, ref, "empty category")
    assert np.isnan(got[0][0, 1]) and not np.isnan(got[0][0, 0])


@pytest.mark.parametrize("shape", [(1, 1, 1), (3, 2, 5), (0, 2, 3), (64, 33, 65), (5000, 1, 1)])
def test_ragged_shapes(gpu_device, shape):
    import synth
    S, FC, FQ = shape
    print(f"groups shape {shape}", flush=True)
    L, X = synth.categorical_continuous(max(S, 1), FC, FQ, 3, missing=0.2, seed=S + FC + FQ)
    L, X = L[:S], X[:S]
    D = np.where(np.isnan(L), np.nan, L >= 1).astype(np.float32)  # dichotomous labels
    _check(_run_gpu("ttest", D, X, gpu_device, welch=True), og.ttest(D, X, welch=True), f"ttest {shape}")
    _check(_run_gpu("anova", L, X, gpu_device, ncat=3), og.anova(L, X, ncat=3), f"anova {shape}")


def test_sentinel(gpu_device):
    import synth
    print("groups sentinel", flush=True)
    L, X = synth.categorical_continuous(400, 5, 9, 3, seed=21)
    Ls = np.where(np.isnan(L), -7.0, L).astype(np.float32)
    Xs = np.where(np.isnan(X), -7.0, X).astype(np.float32)
    got = _run_gpu("anova", Ls, Xs, gpu_device, ncat=3, missing=-7.0)
    _check(got, og.anova(L, X, ncat=3), "sentinel")


@pytest.mark.parametrize("kind", ["ttest", "anova"])
def test_full_size_sampled_pairs(gpu_device, kind):
    """10,000 samples, 30% missing on both sides (the headline's sample count
    and missingness); the oracle checks 400 seeded pairs of the full output."""
    import synth
    print(f"groups full size {kind}", flush=True)
    ncat = 2 if kind == "ttest" else 4
    FC, FQ = (96, 1000) if kind == "ttest" else (48, 700)
    L, X = synth.categorical_continuous(10_000, FC, FQ, ncat, seed=31)
    kw = {"welch": True} if kind == "ttest" else {"ncat": ncat}
    s, p, n = _run_gpu(kind, L, X, gpu_device, **kw)
    rng = np.random.default_rng(5)
    pairs = list(zip(rng.integers(0, FC, 400).tolist(), rng.integers(0, FQ, 400).tolist()))
    if kind == "ttest":
        rs, rp, rn = og.ttest(L, X, welch=True, pairs=pairs)
    else:
        rs, rp, rn = og.anova(L, X, ncat=ncat, pairs=pairs)
    gi = np.array([a for a, _ in pairs])
    hi = np.array([b for _, b in pairs])
    _check((s[gi, hi], p[gi, hi], n[gi, hi]), (rs, rp, rn), f"{kind} full size")
    # an effect is present in some pairs (the generator shifts a third of the
    # continuous columns by their source label)
    assert np.nanmin(p) < 1e-10
