"""GPU parity of the rank tests (napy_mannwhitney, napy_kruskal) against the
FP64 oracle (oracle/ranktests.py) on seeded synthetic inputs.

Ranks are exact on both sides (integers and halves), so U and n must match
exactly.  The oracle forms H as 12 / (n (n + 1)) sum R_k^2 / n_k - 3 (n + 1),
which loses about n * 1e-16 absolute to cancellation, the device the
cancellation-free sum of squared deviations; H agrees to 1e-9 relative plus
1e-8 absolute.  The asymptotic p-values come from SciPy's normal and
chi-squared tails on the oracle's side and from the device's erfc and
incomplete gamma (pinned at 1e-12 against a 40-digit reference in
test_abi.py), so p agrees to 1e-8 relative; exact p-values are ratios of the
same counts (1e-10).  NaN placement must match exactly.
"""

import numpy as np
import pytest

from oracle import ranktests as orank

pytestmark = pytest.mark.gpu


def _run(kind, L, X, gpu_device, **kw):
    import torch
    import paper_2505_00448_amd as napy
    Lt = torch.from_numpy(np.ascontiguousarray(L)).to(gpu_device)
    Xt = torch.from_numpy(np.ascontiguousarray(X)).to(gpu_device)
    out = napy.mannwhitney(Lt, Xt, **kw) if kind == "mwu" else napy.kruskal(Lt, Xt, **kw)
    key = "U" if kind == "mwu" else "H"
    return out[key].cpu().numpy(), out["p"].cpu().numpy(), out["n"].cpu().numpy()


def _check(kind, got, ref, what):
    s, p, n = got
    rs, rp, rn = ref
    assert np.array_equal(np.isnan(s), np.isnan(rs)), f"{what}: NaN placement of the statistic differs"
    assert np.array_equal(np.isnan(p), np.isnan(rp)), f"{what}: NaN placement of p differs"
    ok = ~np.isnan(rs)
    if kind == "mwu":
        np.testing.assert_array_equal(s[ok], rs[ok], err_msg=f"{what} U")
    else:
        np.testing.assert_allclose(s[ok], rs[ok], rtol=1e-9, atol=1e-8, err_msg=f"{what} H")
    ok = ~np.isnan(rp)
    np.testing.assert_allclose(p[ok], rp[ok], rtol=1e-8, atol=1e-300, err_msg=f"{what} p")
    np.testing.assert_array_equal(n, rn, err_msg=f"{what} n")


def _edges(L, X, ncat, rng):
    """Degenerate columns: one group only, an out-of-range label, a
    non-integer label, all missing; continuous columns tied everywhere, with
    heavy ties (three values) and all missing."""
    S = L.shape[0]
    one_group = np.where(np.isnan(L[:, 0]), np.nan, 0.0)
    out_of_range = L[:, 0].copy()
    out_of_range[3] = ncat
    non_int = L[:, 0].copy()
    non_int[4] = 0.5
    L2 = np.column_stack([L, one_group, out_of_range, non_int, np.full(S, np.nan)]).astype(np.float32)
    const = np.full(S, 3.25)
    const[rng.random(S) < 0.2] = np.nan
    three = rng.integers(0, 3, S).astype(np.float64)
    three[rng.random(S) < 0.1] = np.nan
    X2 = np.column_stack([X, const, three, np.full(S, np.nan)]).astype(np.float32)
    return L2, X2


@pytest.mark.parametrize("mode", ["auto", "asymptotic"])
def test_mannwhitney_matches_oracle(gpu_device, mode):
    import synth
    print(f"mannwhitney mode={mode}", flush=True)
    rng = np.random.default_rng(3)
    L, X = synth.categorical_continuous(901, 11, 140, 2, seed=41)
    X[:, :40] = np.round(X[:, :40], 1)  # columns with many ties
    L, X = _edges(L, X, 2, rng)
    got = _run("mwu", L, X, gpu_device, mode=mode)
    ref = orank.mannwhitney(L, X, mode=mode)
    _check("mwu", got, ref, f"mwu {mode}")
    FC, FQ = L.shape[1], X.shape[1]
    assert np.all(np.isnan(got[0][FC - 4])) and np.all(got[2][FC - 3] == 0) and np.all(got[2][FC - 2] == 0)
    assert np.all(got[1][:FC - 4, FQ - 3] == 1.0)  # every value tied: s = 0, p = 1


def test_mannwhitney_exact_pairs(gpu_device):
    """Small groups without ties: the exact distribution.  Columns with a
    rare label (2 .. 9 samples) against tie-free continuous columns, at 60
    samples and at 10,000 (the generating function up to degree 35,000)."""
    print("mannwhitney exact", flush=True)
    rng = np.random.default_rng(17)
    for S in (60, 10_000):
        FC, FQ = 9, 12
        L = np.zeros((S, FC))
        for j in range(FC):
            L[rng.choice(S, j + 2, replace=False), j] = 1.0
        L[rng.random((S, FC)) < 0.05] = np.nan
        X = np.column_stack([rng.permutation(S) for _ in range(FQ)]).astype(np.float64)
        X[rng.random((S, FQ)) < 0.05] = np.nan
        X[:, 0] = np.round(X[:, 0] / 3.0)  # one tied column: asymptotic
        L, X = L.astype(np.float32), X.astype(np.float32)
        got = _run("mwu", L, X, gpu_device, mode="auto")
        ref = orank.mannwhitney(L, X, mode="auto")
        _check("mwu", got, ref, f"mwu exact S={S}")
        n1 = np.array([[np.sum((L[:, j] == 1) & ~np.isnan(X[:, h])) for h in range(FQ)] for j in range(FC)])
        assert np.sum(n1[:, 1:] < 8) > 40  # most untied pairs took the exact branch


def test_mannwhitney_many_exact_pairs(gpu_device):
    """Tiny samples: nearly every pair is exact (more pairs than the exact
    kernel's workgroups)."""
    print("mannwhitney many exact", flush=True)
    rng = np.random.default_rng(23)
    S, FC, FQ = 14, 30, 40
    L = rng.integers(0, 2, (S, FC)).astype(np.float32)
    X = rng.normal(size=(S, FQ)).astype(np.float32)
    L[rng.random((S, FC)) < 0.1] = np.nan
    X[rng.random((S, FQ)) < 0.1] = np.nan
    _check("mwu", _run("mwu", L, X, gpu_device), orank.mannwhitney(L, X), "many exact")


def test_tie_patterns(gpu_device):
    """Tie runs handled each way the library chooses: a few short runs (pairs
    and triples, some across 64-position chunks), the same plus one long
    run, many medium runs, and no ties."""
    print("rank tests tie patterns", flush=True)
    rng = np.random.default_rng(29)
    S = 3000
    cols = []
    for kind in range(12):
        x = rng.permutation(S).astype(np.float64)
        if kind % 4 == 0:
            for _ in range(25):
                a, b = rng.choice(S, 2, replace=False)
                x[b] = x[a]
            t = rng.choice(S, 3, replace=False)
            x[t] = x[t[0]]
        elif kind % 4 == 1:
            for _ in range(10):
                a, b = rng.choice(S, 2, replace=False)
                x[b] = x[a]
            x[rng.choice(S, 300, replace=False)] = -1.0
        elif kind % 4 == 2:
            x = np.floor(x / 37.0)
        cols.append(x)
    X = np.column_stack(cols)
    X[rng.random(X.shape) < 0.05] = np.nan
    X = X.astype(np.float32)
    L = rng.integers(0, 3, (S, 7)).astype(np.float32)
    L[rng.random(L.shape) < 0.1] = np.nan
    D = np.where(np.isnan(L), np.nan, L >= 1).astype(np.float32)
    _check("mwu", _run("mwu", D, X, gpu_device), orank.mannwhitney(D, X), "tie patterns mwu")
    _check("kw", _run("kw", L, X, gpu_device, ncat=3), orank.kruskal(L, X, ncat=3), "tie patterns kruskal")


@pytest.mark.parametrize("ncat", [3, 5, 9, 17])
def test_kruskal_matches_oracle(gpu_device, ncat):
    import synth
    print(f"kruskal ncat={ncat}", flush=True)
    rng = np.random.default_rng(ncat)
    L, X = synth.categorical_continuous(1203, 9, 75, ncat, seed=ncat + 50)
    X[:, ::3] = np.round(X[:, ::3], 1)
    L, X = _edges(L, X, ncat, rng)
    got = _run("kw", L, X, gpu_device, ncat=ncat)
    ref = orank.kruskal(L, X, ncat=ncat)
    _check("kw", got, ref, f"kruskal ncat={ncat}")
    FC, FQ = L.shape[1], X.shape[1]
    assert np.all(np.isnan(got[0][:FC - 4, FQ - 3]))  # every value tied
    assert np.all(np.isnan(got[0][FC - 4]))  # one category


def test_kruskal_empty_category_within_pair(gpu_device):
    print("kruskal empty category", flush=True)
    rng = np.random.default_rng(8)
    S = 300
    L = rng.integers(0, 3, size=(S, 2)).astype(np.float32)
    X = rng.normal(size=(S, 3)).astype(np.float32)
    X[L[:, 0] == 2, 1] = np.nan
    got = _run("kw", L, X, gpu_device, ncat=3)
    _check("kw", got, orank.kruskal(L, X, ncat=3), "empty category")
    assert np.isnan(got[0][0, 1]) and not np.isnan(got[0][0, 0])


@pytest.mark.parametrize("shape", [(1, 1, 1), (3, 2, 5), (0, 2, 3), (64, 33, 65), (130, 1, 9), (5000, 2, 1)])
def test_ragged_shapes(gpu_device, shape):
    import synth
    S, FC, FQ = shape
    print(f"rank tests shape {shape}", flush=True)
    L, X = synth.categorical_continuous(max(S, 1), FC, FQ, 3, missing=0.2, seed=S + FC + FQ)
    L, X = L[:S], X[:S]
    D = np.where(np.isnan(L), np.nan, L >= 1).astype(np.float32)
    _check("mwu", _run("mwu", D, X, gpu_device), orank.mannwhitney(D, X), f"mwu {shape}")
    _check("kw", _run("kw", L, X, gpu_device, ncat=3), orank.kruskal(L, X, ncat=3), f"kruskal {shape}")


def test_sentinel_and_default_ncat(gpu_device):
    import synth
    print("rank tests sentinel", flush=True)
    L, X = synth.categorical_continuous(400, 5, 9, 4, seed=21)
    Ls = np.where(np.isnan(L), -7.0, L).astype(np.float32)
    Xs = np.where(np.isnan(X), -7.0, X).astype(np.float32)
    _check("kw", _run("kw", Ls, Xs, gpu_device, missing=-7.0), orank.kruskal(L, X), "sentinel")


@pytest.mark.parametrize("S", [24576, 24577, 50000, 65535])
def test_max_samples(gpu_device, S):
    """The largest column the LDS sort takes (24,576), one sample more (the
    global-memory sort), 50,000 and the 16-bit limit 65,535 (labels read from
    global memory, 64-bit rank sums): untied, grouped and densely tied
    continuous columns, one complete; labels with and without missing."""
    print(f"rank tests max samples S={S}", flush=True)
    rng = np.random.default_rng(88 + S)
    X = np.column_stack([rng.standard_normal(S), rng.poisson(4, S), np.round(rng.standard_normal(S), 1),
                         rng.permutation(S)]).astype(np.float64)
    X[rng.random(X.shape) < 0.3] = np.nan
    X[:, 3] = rng.permutation(S)
    L = rng.integers(0, 3, (S, 3)).astype(np.float64)
    L[rng.random(L.shape) < 0.2] = np.nan
    L[:, 2] = rng.integers(0, 3, S)
    X, L = X.astype(np.float32), L.astype(np.float32)
    D = np.where(np.isnan(L), np.nan, L >= 1).astype(np.float32)
    _check("mwu", _run("mwu", D, X, gpu_device), orank.mannwhitney(D, X), "mwu max samples")
    _check("kw", _run("kw", L, X, gpu_device, ncat=3), orank.kruskal(L, X, ncat=3), "kruskal max samples")


@pytest.mark.parametrize("kind", ["mwu", "kw"])
def test_full_size_sampled_pairs(gpu_device, kind):
    """10,000 samples, 30% missing on both sides; the oracle checks 300
    seeded pairs of the full output."""
    import synth
    print(f"rank tests full size {kind}", flush=True)
    ncat = 2 if kind == "mwu" else 4
    FC, FQ = (64, 1000) if kind == "mwu" else (40, 600)
    L, X = synth.categorical_continuous(10_000, FC, FQ, ncat, seed=33)
    X[:, ::4] = np.round(X[:, ::4], 1)
    s, p, n = _run(kind, L, X, gpu_device, **({} if kind == "mwu" else {"ncat": ncat}))
    rng = np.random.default_rng(6)
    pairs = list(zip(rng.integers(0, FC, 300).tolist(), rng.integers(0, FQ, 300).tolist()))
    if kind == "mwu":
        ref = orank.mannwhitney(L, X, pairs=pairs)
    else:
        ref = orank.kruskal(L, X, ncat=ncat, pairs=pairs)
    gi = np.array([a for a, _ in pairs])
    hi = np.array([b for _, b in pairs])
    _check(kind, (s[gi, hi], p[gi, hi], n[gi, hi]), ref, f"{kind} full size")
    assert np.nanmin(p) < 1e-10
