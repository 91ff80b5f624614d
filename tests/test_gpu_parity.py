"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle on the
same seeded inputs.

Bars: counts and ranks bit-exact; Pearson |dr| <= 1e-6 (FP32, BF16x3) and
<= 1e-12 (FP64 validation mode); Spearman |drho| <= 1e-12; NaN placement
exact; p through its conditioning (tests/parity_util.py).
"""

import math

import numpy as np
import pytest

import synth
from oracle import oracle as orc
from parity_util import assert_counts_equal, assert_p_close, assert_r_close

pytestmark = pytest.mark.gpu

R_TOL = {"fp32": 1e-6, "bf16x3": 1e-6, "fp64": 1e-12}


def _napy():
    import paper_2505_00448_amd as napy
    return napy


def _to_dev(X, dev):
    import torch
    return torch.from_numpy(np.ascontiguousarray(X, dtype=np.float32)).to(dev)


def _np(t):
    return t.detach().cpu().numpy()


def _run(method, X, dev, precision="fp32", missing=None):
    napy = _napy()
    Xd = _to_dev(X, dev)
    if method == "pearson":
        out = napy.pearson(Xd, precision=precision, missing=missing)
    else:
        out = napy.spearman(Xd, missing=missing)
    return _np(out["r"]), _np(out["p"]), _np(out["n"])


def _check_full(method, X, dev, precision="fp32", missing=None, where=""):
    r, p, n = _run(method, X, dev, precision, missing)
    if method == "pearson":
        ro, po, no = orc.pearson(X, missing=missing)
        tol = R_TOL[precision]
    else:
        ro, po, no = orc.spearman(X, missing=missing)
        tol = 1e-12
    assert_counts_equal(n, no, where)
    worst = assert_r_close(r, ro, tol, where)
    assert_p_close(p, po, ro, no, max(worst, 1e-15), where)
    assert np.array_equal(r, r.T, equal_nan=True), f"{where}: r not symmetric"
    return worst


# ---------------------------------------------------------------------------
# small configuration (500 x 50), all methods and precisions
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("precision", ["fp32", "bf16x3", "fp64"])
def test_pearson_small(gpu_device, precision):
    X = synth.cfg_plain_small()
    _check_full("pearson", X, gpu_device, precision, where=f"pearson-500x50-{precision}")


def test_spearman_small(gpu_device):
    X = synth.cfg_plain_small()
    _check_full("spearman", X, gpu_device, where="spearman-500x50")


def test_spearman_heavy_ties(gpu_device):
    X = synth.heavy_ties(700, 40, levels=5, missing=0.2)
    _check_full("spearman", X, gpu_device, where="spearman-heavy-ties")


@pytest.mark.parametrize("method", ["pearson", "spearman"])
def test_edge_matrix(gpu_device, method):
    X = synth.edge_matrix()
    precisions = ["fp32", "bf16x3", "fp64"] if method == "pearson" else ["fp32"]
    for prec in precisions:
        _check_full(method, X, gpu_device, prec, where=f"edge-{method}-{prec}")


# ---------------------------------------------------------------------------
# ragged shapes: several tiles, partial tiles, tiny and empty inputs
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("S,F", [(1, 3), (2, 5), (3, 1), (0, 4), (15, 9), (16, 7), (17, 33), (31, 70), (777, 130),
                                 (1500, 65), (64, 64), (65, 129)])
def test_ragged_shapes(gpu_device, S, F):
    rng = np.random.default_rng(S * 1000 + F)
    X = rng.standard_normal((S, F)).astype(np.float32)
    if S:
        X[rng.random((S, F)) < 0.25] = np.nan
    for prec in ("fp32", "bf16x3", "fp64"):
        _check_full("pearson", X, gpu_device, prec, where=f"ragged-pearson-{S}x{F}-{prec}")
    _check_full("spearman", X, gpu_device, where=f"ragged-spearman-{S}x{F}")


def test_paper_shape(gpu_device):
    X = synth.paper_shape(250, 250)
    _check_full("pearson", X, gpu_device, "fp32", where="paper-shape-pearson")
    _check_full("pearson", X, gpu_device, "bf16x3", where="paper-shape-pearson-bf16x3")
    _check_full("spearman", X, gpu_device, where="paper-shape-spearman")


def test_sentinel_missing_value(gpu_device):
    X = synth.cfg_plain_small(F=20)
    Xs = np.where(np.isnan(X), np.float32(-999.0), X).astype(np.float32)
    for method in ("pearson", "spearman"):
        r1, p1, n1 = _run(method, X, gpu_device)
        r2, p2, n2 = _run(method, Xs, gpu_device, missing=-999.0)
        assert np.array_equal(n1, n2)
        assert np.array_equal(r1, r2, equal_nan=True)


def test_signed_zero_and_constant_subsets(gpu_device):
    rng = np.random.default_rng(1)
    S = 300
    x = rng.standard_normal(S).astype(np.float32)
    zeros = np.where(rng.random(S) < 0.5, np.float32(0.0), np.float32(-0.0))
    const_on_subset = np.where(np.arange(S) < 150, np.float32(2.0), x)
    binary = (rng.random(S) < 0.5).astype(np.float32)
    pois = rng.poisson(4, S).astype(np.float32)
    X = np.stack([x, zeros, const_on_subset, binary, pois, -x], axis=1)
    miss = np.zeros_like(X, dtype=bool)
    miss[150:, 0] = True  # column 0 only present where column 2 is constant
    X[miss] = np.nan
    for prec in ("fp32", "bf16x3", "fp64"):
        _check_full("pearson", X, gpu_device, prec, where=f"constant-subsets-{prec}")
    _check_full("spearman", X, gpu_device, where="constant-subsets-spearman")


# ---------------------------------------------------------------------------
# ranks, bit-exact
# ---------------------------------------------------------------------------

def test_pair_ranks_bit_exact(gpu_device):
    napy = _napy()
    X = np.concatenate([synth.heavy_ties(900, 6, levels=4, missing=0.3),
                        synth.cfg_plain_small(S=900, F=6)], axis=1)
    Xd = _to_dev(X, gpu_device)
    for g, h in [(0, 1), (2, 7), (8, 9), (3, 3), (11, 4), (6, 10)]:
        rg, rh = napy.spearman_pair_ranks(Xd, g, h)
        og, oh, n = orc.pair_ranks(X, g, h)
        exp_g = np.where(np.isnan(og), -1, np.round(2 * np.nan_to_num(og))).astype(np.int64)
        exp_h = np.where(np.isnan(oh), -1, np.round(2 * np.nan_to_num(oh))).astype(np.int64)
        assert np.array_equal(_np(rg).astype(np.int64), exp_g), (g, h)
        assert np.array_equal(_np(rh).astype(np.int64), exp_h), (g, h)


# ---------------------------------------------------------------------------
# p-value routine at the GPU's own (r, n)
# ---------------------------------------------------------------------------

def test_device_pvalue_against_mpmath(gpu_device):
    import torch
    napy = _napy()
    rng = np.random.default_rng(5)
    ns = np.array([3, 4, 5, 7, 10, 37, 100, 1000, 3500, 6650, 10000, 20000, 24576] * 12, dtype=np.int32)
    rs = np.concatenate([rng.uniform(-0.999, 0.999, ns.size // 2),
                         rng.uniform(-0.05, 0.05, ns.size - ns.size // 2)])
    p = _np(napy.pvalue_device(torch.from_numpy(rs).to(gpu_device), torch.from_numpy(ns).to(gpu_device)))
    for r, n, pv in zip(rs, ns, p):
        ref = orc.pvalue_mp(float(r), int(n))
        if ref < 1e-300:
            assert pv < 1e-290
        else:
            assert abs(pv - ref) <= 1e-10 * ref, (r, n, pv, ref)
    # closed forms
    p3 = _np(napy.pvalue_device(torch.tensor([0.3, -0.8], dtype=torch.float64, device=gpu_device),
                                torch.tensor([3, 4], dtype=torch.int32, device=gpu_device)))
    assert abs(p3[0] - (1 - 2 / math.pi * math.asin(0.3))) <= 1e-13
    assert abs(p3[1] - 0.2) <= 1e-13


# ---------------------------------------------------------------------------
# determinism and subset queries
# ---------------------------------------------------------------------------

def test_bitwise_determinism(gpu_device):
    X = synth.cfg_gpu_headline(S=3000, F=200)
    for method, prec in (("pearson", "fp32"), ("pearson", "bf16x3"), ("spearman", "fp32")):
        a = _run(method, X, gpu_device, prec)
        b = _run(method, X, gpu_device, prec)
        for u, v in zip(a, b):
            assert np.array_equal(u, v, equal_nan=True), (method, prec)


@pytest.mark.parametrize("F,pad,offset", [(64, 4, 0), (70, 4, 0), (70, 3, 0), (64, 4, 1), (130, 0, 1)])
def test_padded_and_unaligned_rows(gpu_device, F, pad, offset):
    """X handed over as a view of a wider buffer: leading dimension F + pad,
    first element `offset` floats into it (16-byte aligned rows and a
    multiple-of-4 leading dimension take the key transpose's vector loads,
    the rest its element loads).  Results bit-identical to the contiguous
    call, which the oracle pins."""
    import torch
    napy = _napy()
    S = 300
    X = synth.heavy_ties(S, F, levels=7, missing=0.2, seed=77)
    X[:, : F // 2] = synth.cfg_plain_small(S=S, F=F // 2)
    print(f"[padded] F={F} pad={pad} offset={offset}", flush=True)
    big = torch.full((S, F + pad + offset), 123.0, dtype=torch.float32, device=gpu_device)
    big[:, offset:offset + F] = torch.from_numpy(X).to(gpu_device)
    view = big[:, offset:offset + F]
    assert view.stride(0) == F + pad + offset
    for method in ("spearman", "pearson"):
        got = napy.spearman(view) if method == "spearman" else napy.pearson(view, precision="fp32")
        ref = _run(method, X, gpu_device)
        for k, want in zip(("r", "p", "n"), ref):
            assert np.array_equal(_np(got[k]), want, equal_nan=True), (method, k)
    _check_full("spearman", X, gpu_device, where=f"padded-{F}-{pad}-{offset}")


def test_subset_queries_match_full_calls(gpu_device):
    import torch
    napy = _napy()
    X = synth.cfg_serving_base(S=2000, F=150)
    Xd = _to_dev(X, gpu_device)
    base = napy.SpearmanBase(Xd)
    rng = np.random.default_rng(3)
    for trial in range(4):
        rows = np.sort(rng.choice(2000, size=int(rng.integers(50, 1900)), replace=False)).astype(np.int32)
        cols = rng.choice(150, size=int(rng.integers(2, 150)), replace=False).astype(np.int32)
        rt = torch.from_numpy(rows).to(gpu_device)
        ct = torch.from_numpy(cols).to(gpu_device)
        sub = X[np.ix_(rows, cols)]
        for prec in ("fp32", "bf16x3"):
            got = napy.pearson_subset(Xd, rt, ct, precision=prec)
            ref = napy.pearson(_to_dev(sub, gpu_device), precision=prec)
            for k in ("r", "p", "n"):
                assert np.array_equal(_np(got[k]), _np(ref[k]), equal_nan=True), (trial, prec, k)
        got = base.subset(rt, ct)
        ref = napy.spearman(_to_dev(sub, gpu_device))
        for k in ("r", "p", "n"):
            assert np.array_equal(_np(got[k]), _np(ref[k]), equal_nan=True), (trial, "spearman", k)
        # and against the oracle
        ro, po, no = orc.spearman(sub)
        assert_counts_equal(_np(got["n"]), no, "subset-spearman")
        assert_r_close(_np(got["r"]), ro, 1e-12, "subset-spearman")


def test_subset_queries_with_ties(gpu_device):
    """Subset queries on a base with tie runs of every kind: few levels, long
    runs, scattered pairs, a constant column.  Row subsets shrink runs to one
    sample or empty them; the result must equal the full call on the
    submatrix bit for bit, and the oracle."""
    import torch
    napy = _napy()
    S = 2500
    rng = np.random.default_rng(44)
    X = np.concatenate([synth.heavy_ties(S, 6, levels=3, seed=7), synth.heavy_ties(S, 6, levels=40, seed=8),
                        synth.cfg_serving_base(S=S, F=6)], axis=1).astype(np.float64)
    for j in range(12, 18):
        for _ in range(30):  # scattered duplicate pairs in continuous columns
            a, b = rng.choice(S, 2, replace=False)
            X[b, j] = X[a, j]
    X = np.column_stack([X, np.full(S, 1.5)]).astype(np.float32)
    Xd = _to_dev(X, gpu_device)
    base = napy.SpearmanBase(Xd)
    F = X.shape[1]
    for trial, frac in enumerate((0.02, 0.3, 0.9, 1.0)):
        rows = np.sort(rng.choice(S, size=max(3, int(frac * S)), replace=False)).astype(np.int32)
        cols = rng.permutation(F)[: max(2, F - 3 * trial)].astype(np.int32)
        print(f"subset with ties trial {trial}: {rows.size} rows, {cols.size} columns", flush=True)
        got = base.subset(torch.from_numpy(rows).to(gpu_device), torch.from_numpy(cols).to(gpu_device))
        sub = X[np.ix_(rows, cols)]
        ref = napy.spearman(_to_dev(sub, gpu_device))
        for k in ("r", "p", "n"):
            assert np.array_equal(_np(got[k]), _np(ref[k]), equal_nan=True), (trial, k)
        ro, po, no = orc.spearman(sub)
        assert_counts_equal(_np(got["n"]), no, "subset-ties")
        assert_r_close(_np(got["r"]), ro, 1e-12, "subset-ties")


# ---------------------------------------------------------------------------
# complete samples far from the column mean (value-dependent missingness)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("precision", ["fp32", "bf16x3", "fp64"])
def test_mode_selected_partners(gpu_device, precision):
    """Bimodal columns whose partners are observed on one mode only: the
    pair's complete samples lie 10, 100 and 1,000 of their own sds from the
    column's observed mean, where sums about the column mean cancel; and
    partners constant on that mode (exact NaN)."""
    X = synth.mode_selected()
    _check_full("pearson", X, gpu_device, precision, where=f"mode-selected-{precision}")


# ---------------------------------------------------------------------------
# full-size headline configuration (10,000 x 1,000): every pair against the
# oracle
# ---------------------------------------------------------------------------

@pytest.fixture(scope="module")
def headline():
    return synth.cfg_gpu_headline()


@pytest.fixture(scope="module")
def headline_oracle(headline):
    cache = {}

    def get(method):
        if method not in cache:
            print(f"[headline oracle] {method}, all pairs of 10,000 x 1,000", flush=True)
            cache[method] = orc.pearson(headline) if method == "pearson" else orc.spearman(headline)
        return cache[method]
    return get


def _sample_pairs(F, k, seed):
    rng = np.random.default_rng(seed)
    g = rng.integers(0, F, k)
    h = rng.integers(0, F, k)
    d = np.arange(0, F, max(1, F // 50))
    return np.concatenate([g, d]), np.concatenate([h, d])


@pytest.mark.parametrize("method,precision", [("pearson", "fp32"), ("pearson", "bf16x3"),
                                              ("pearson", "fp64"), ("spearman", "fp32")])
def test_headline_full_size(gpu_device, headline, headline_oracle, method, precision):
    """All F (F + 1) / 2 pairs of the headline matrix, element by element:
    counts bit-exact, r within the precision's bar, NaN placement exact, p
    through its conditioning."""
    X = headline
    print(f"[headline] {method} {precision}", flush=True)
    r, p, n = _run(method, X, gpu_device, precision)
    ro, po, no = headline_oracle(method)
    tol = R_TOL[precision] if method == "pearson" else 1e-12
    where = f"headline-{method}-{precision}"
    assert_counts_equal(n, no, where)
    worst = assert_r_close(r, ro, tol, where)
    assert_p_close(p, po, ro, no, max(worst, 1e-15), where)
    assert np.array_equal(r, r.T, equal_nan=True)
    print(f"[headline] {method} {precision}: max |dr| = {worst:.3e} over {r.size} entries", flush=True)


# ---------------------------------------------------------------------------
# precision form at full size (50,000 x 4,000, column means up to 1e5)
# ---------------------------------------------------------------------------

@pytest.fixture(scope="module")
def precision_case():
    X = synth.cfg_precision()
    M = (~np.isnan(X)).astype(np.float32)
    # 0/1 products summed in float32 stay exact below 2**24
    N = (M.T @ M).astype(np.int64)
    return X, N


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
def test_precision_form_full_size(gpu_device, precision_case, precision):
    X, N = precision_case
    S, F = X.shape
    print(f"[precision-form] {S}x{F} {precision}", flush=True)
    r, p, n = _run("pearson", X, gpu_device, precision)
    where = f"precision-form-{precision}"
    assert_counts_equal(n, N, where + "-full-n")
    assert np.array_equal(r, r.T, equal_nan=True)
    assert np.nanmax(np.abs(r)) <= 1.0
    gi, hi = _sample_pairs(F, 1500, 29)
    ro, po, no = orc.pearson_pairs(X, gi, hi)
    worst = assert_r_close(r[gi, hi], ro, 1e-6, where)
    assert_p_close(p[gi, hi], po, ro, no, max(worst, 1e-15), where)


# ---------------------------------------------------------------------------
# tie runs of every length and position relative to the 64-position chunks
# ---------------------------------------------------------------------------

def _tie_stress_matrix(S=3000, seed=21):
    rng = np.random.default_rng(seed)
    cols = []
    cols.append(rng.integers(0, 3, S).astype(np.float32))             # 3 huge runs
    cols.append(rng.integers(0, 40, S).astype(np.float32))            # runs ~75 long
    x = rng.standard_normal(S).astype(np.float32)
    dup = x.copy()
    idx = rng.choice(S, 200, replace=False)
    dup[idx] = dup[rng.choice(S, 200, replace=False)]                  # scattered pairs/triples
    cols.append(dup)
    cols.append(np.round(rng.standard_normal(S) * 4).astype(np.float32))  # ~30 levels
    cols.append(x)                                                     # no ties
    cols.append((rng.integers(0, 2, S) * 2 - 1).astype(np.float32) * 0.0)  # all (+-)0: one run
    X = np.stack(cols, axis=1)
    X[rng.random(X.shape) < 0.35] = np.nan
    X[rng.random(S) < 0.5, 1] = np.nan                                 # sparse kept in column 1
    return X


def test_tie_runs_across_chunks(gpu_device):
    X = _tie_stress_matrix()
    _check_full("spearman", X, gpu_device, where="tie-stress")


def _grouped_matrix(S=1024, seed=31):
    """Columns of few value groups (tie runs plus untied values, at most a
    couple of dozen), with observed counts that are exact multiples of 64 and
    256, next to untied columns and columns with a few duplicate pairs."""
    rng = np.random.default_rng(seed)

    def observe(x, count):
        x = x.astype(np.float64)
        x[rng.permutation(S)[count:]] = np.nan
        return x

    cols = [observe(rng.poisson(3, S), 256), observe(rng.poisson(4, S), 512), observe(rng.poisson(2, S), 640),
            rng.poisson(4, S).astype(np.float64)]
    few = rng.integers(0, 6, S).astype(np.float64)
    few[rng.choice(S, 3, replace=False)] = [100.0, 101.5, -7.0]  # three untied values
    cols.append(observe(few, 700))
    cols.append(observe(rng.integers(0, 15, S), 900))
    x = rng.standard_normal(S)
    cols.append(observe(x, 716))
    d = rng.standard_normal(S)
    for _ in range(4):
        a, b = rng.choice(S, 2, replace=False)
        d[b] = d[a]
    cols.append(observe(d, 830))
    return np.column_stack(cols).astype(np.float32)


def test_grouped_columns(gpu_device):
    X = _grouped_matrix()
    _check_full("spearman", X, gpu_device, where="grouped-columns")


def _value_groups(col):
    """(tie runs, untied values) among a column's observed values."""
    v = col[~np.isnan(col)]
    _, counts = np.unique(v, return_counts=True)
    return int((counts > 1).sum()), int((counts == 1).sum())


def test_grouped_limit_23_groups(gpu_device):
    """Columns at the grouped limit: exactly 23 value groups (tie runs plus
    untied values), whose run-rank indices 0..22 sit next to the index 23 of
    the table's zero entry that codes a missing sample; a column of 24
    groups just past the limit; untied and sparsely tied partners; missing
    values throughout, S = 1,000 (several walk groups and a ragged tail)."""
    rng = np.random.default_rng(2323)
    S = 1000

    def runs_plus_singletons(nruns, singles):
        x = rng.integers(0, nruns, S).astype(np.float64)
        idx = rng.choice(S, len(singles), replace=False)
        x[idx] = singles
        return x, idx

    c0, k0 = runs_plus_singletons(22, [99.0])                # 22 runs + 1 untied value
    c1, k1 = runs_plus_singletons(23, [])                    # 23 runs
    c2, k2 = runs_plus_singletons(21, [-5.0, 77.5])          # 21 runs + 2 untied values
    c3, k3 = runs_plus_singletons(24, [])                    # 24 runs: past the limit
    c4 = rng.standard_normal(S)                              # untied
    c5 = rng.standard_normal(S)
    for _ in range(3):                                       # a few duplicated pairs
        a, b = rng.choice(S, 2, replace=False)
        c5[b] = c5[a]
    c6, k6 = runs_plus_singletons(23, [])                    # 23 runs, complete
    X = np.column_stack([c0, c1, c2, c3, c4, c5, c6])
    miss = rng.random(X.shape) < 0.3
    miss[:, 6] = False
    for j, keep in ((0, k0), (2, k2)):
        miss[keep, j] = False                                # the untied values stay observed
    X[miss] = np.nan
    groups = [sum(_value_groups(X[:, j])) for j in range(X.shape[1])]
    assert groups[0] == groups[1] == groups[2] == groups[6] == 23 and groups[3] == 24, groups
    _check_full("spearman", X.astype(np.float32), gpu_device, where="grouped-limit-23")


def test_spearman_max_samples(gpu_device):
    """S = 24,576, the largest sample count the 16-bit sorted orders hold:
    untied, sparsely tied, grouped (few values) and densely tied columns,
    one of them complete (positions and run ends up to 24,576)."""
    rng = np.random.default_rng(77)
    S = 24576
    cols = [rng.standard_normal(S), rng.poisson(4, S).astype(np.float64), np.round(rng.standard_normal(S), 2),
            rng.integers(0, 3, S).astype(np.float64), rng.standard_normal(S)]
    d = rng.standard_normal(S)
    for _ in range(40):
        a, b = rng.choice(S, 2, replace=False)
        d[b] = d[a]
    cols.append(d)
    X = np.column_stack(cols + [rng.standard_normal(S) for _ in range(4)])
    X[rng.random(X.shape) < 0.3] = np.nan
    X[:, 4] = rng.permutation(S)  # complete and untied
    X[:, 3] = rng.integers(0, 3, S)  # complete, three runs, the last ending at S
    _check_full("spearman", X.astype(np.float32), gpu_device, where="spearman-max-samples")


def _long_columns(S, seed):
    """Columns longer than the LDS sort takes: untied, Poisson, rounded
    normals, grouped (three values, complete, the last run ending at S), a
    complete untied column (positions up to S - 1), one with 40 tied pairs,
    and plain normals; 30% missing elsewhere."""
    rng = np.random.default_rng(seed)
    cols = [rng.standard_normal(S), rng.poisson(4, S).astype(np.float64), np.round(rng.standard_normal(S), 2),
            rng.integers(0, 3, S).astype(np.float64), rng.standard_normal(S)]
    d = rng.standard_normal(S)
    for _ in range(40):
        a, b = rng.choice(S, 2, replace=False)
        d[b] = d[a]
    cols.append(d)
    X = np.column_stack(cols + [rng.standard_normal(S) for _ in range(4)])
    X[rng.random(X.shape) < 0.3] = np.nan
    X[:, 4] = rng.permutation(S)
    X[:, 3] = rng.integers(0, 3, S)
    return X.astype(np.float32)


@pytest.mark.parametrize("S", [24577, 50000, 65535])
def test_spearman_long_columns(gpu_device, S):
    """Above 24,576 samples the columns are sorted in global memory and the
    pair scan reads a's positions (no tie flag) from there: one sample above
    that length, 50,000, and the 16-bit limit 65,535."""
    print(f"[spearman long columns] S={S}", flush=True)
    _check_full("spearman", _long_columns(S, 900 + S), gpu_device, where=f"spearman-long-{S}")


def test_long_columns_ranks_bit_exact(gpu_device):
    """Doubled ranks within I(g, h) at 50,000 samples, bit for bit, for pairs
    of every tie class on either side."""
    napy = _napy()
    X = _long_columns(50000, 4242)
    Xd = _to_dev(X, gpu_device)
    for g, h in [(0, 1), (1, 0), (1, 2), (2, 3), (3, 1), (5, 4), (4, 5), (3, 3), (2, 9)]:
        rg, rh = napy.spearman_pair_ranks(Xd, g, h)
        og, oh, n = orc.pair_ranks(X, g, h)
        exp_g = np.where(np.isnan(og), -1, np.round(2 * np.nan_to_num(og))).astype(np.int64)
        exp_h = np.where(np.isnan(oh), -1, np.round(2 * np.nan_to_num(oh))).astype(np.int64)
        assert np.array_equal(_np(rg).astype(np.int64), exp_g), (g, h, "a side")
        assert np.array_equal(_np(rh).astype(np.int64), exp_h), (g, h, "b side")


def test_tie_runs_ranks_bit_exact(gpu_device):
    napy = _napy()
    X = _tie_stress_matrix(S=1500, seed=5)
    Xd = _to_dev(X, gpu_device)
    F = X.shape[1]
    for g in range(F):
        for h in range(F):
            rg, rh = napy.spearman_pair_ranks(Xd, g, h)
            og, oh, n = orc.pair_ranks(X, g, h)
            exp_g = np.where(np.isnan(og), -1, np.round(2 * np.nan_to_num(og))).astype(np.int64)
            exp_h = np.where(np.isnan(oh), -1, np.round(2 * np.nan_to_num(oh))).astype(np.int64)
            assert np.array_equal(_np(rg).astype(np.int64), exp_g), (g, h, "a side")
            assert np.array_equal(_np(rh).astype(np.int64), exp_h), (g, h, "b side")
