"""Seeded generators for the five workloads and the paper's own simulated shape.

Every generator draws in float64 with numpy's PCG64 and returns float32
samples x variables matrices (row-major, variables contiguous) with NaN for a
missing entry.  The oracle reads the same float32 values promoted to float64.

Workloads (the data are cohort-shaped stand-ins: the paper's cohort data are
access-restricted, so block missingness and integer-valued columns imitate
questionnaire modules and count variables of such a cohort):

* ``cfg_plain_small``   500 x 50, rank-5 Gaussian factor model, 20% MCAR,
                        about 5% of values rounded to one decimal (ties).
* ``cfg_gpu_headline``  10,000 x 1,000, rank-20 factor model, 10% of the
                        columns Poisson(4) integers through a Gaussian copula,
                        30% MCAR plus 100 columns missing on one shared random
                        half of the samples.
* ``cfg_precision``     50,000 x 4,000, column means U(1e3, 1e5) with unit-sd
                        rank-5 factor residuals, 25% MCAR.
* ``cfg_differentiation`` 8,192 x 512, rank-10 factor model, 15% MCAR, with a
                        symmetric N(0,1) loss weight matrix.
* ``cfg_serving_base``  20,000 x 2,000, rank-20 factor model, 30% MCAR, plus a
                        Poisson-arrival query stream (``serving_queries``).
* ``paper_shape``       uniform [0, 1) values with an exact fraction of missing
                        entries per variable, as in the paper's simulated data
                        (Section 4.1.1).
* ``mode_selected``     bimodal columns whose partners are observed on one
                        mode only (missingness that depends on the value), so
                        a pair's complete samples sit many of their own sds
                        away from the column's observed mean.
"""

from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

SEED_BASE = 2505_00448


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def factor_matrix(rng: np.random.Generator, S: int, F: int, rank: int,
                  unit_sd: bool = False, chunk: int = 8192) -> np.ndarray:
    """X = Z L^T + E with Z ~ N(0,1)^{S x rank}, L ~ N(0,1)^{F x rank},
    E ~ N(0,1).  With ``unit_sd`` each column is divided by its model sd
    sqrt(sum_j L_cj^2 + 1).  Returned as float64."""
    L = rng.standard_normal((F, rank))
    out = np.empty((S, F), dtype=np.float64)
    scale = np.sqrt((L * L).sum(axis=1) + 1.0) if unit_sd else None
    for s0 in range(0, S, chunk):
        s1 = min(S, s0 + chunk)
        Z = rng.standard_normal((s1 - s0, rank))
        blk = Z @ L.T
        blk += rng.standard_normal((s1 - s0, F))
        if unit_sd:
            blk /= scale
        out[s0:s1] = blk
    return out


def _mcar(rng: np.random.Generator, X: np.ndarray, frac: float) -> None:
    if frac <= 0:
        return
    S, F = X.shape
    for s0 in range(0, S, 8192):
        s1 = min(S, s0 + 8192)
        m = rng.random((s1 - s0, F)) < frac
        X[s0:s1][m] = np.nan


def cfg_plain_small(seed: int = SEED_BASE + 1, S: int = 500, F: int = 50,
                    missing: float = 0.20, round_frac: float = 0.05) -> np.ndarray:
    rng = _rng(seed)
    X = factor_matrix(rng, S, F, 5)
    r = rng.random((S, F)) < round_frac
    X[r] = np.round(X[r], 1)
    _mcar(rng, X, missing)
    return X.astype(np.float32)


def cfg_gpu_headline(seed: int = SEED_BASE + 2, S: int = 10_000, F: int = 1_000,
                     missing: float = 0.30, n_poisson: int | None = None,
                     n_block: int | None = None, block_frac: float = 0.5) -> np.ndarray:
    from scipy import special, stats
    rng = _rng(seed)
    X = factor_matrix(rng, S, F, 20)
    if n_poisson is None:
        n_poisson = F // 10
    if n_block is None:
        n_block = min(100, F // 10)
    pois_cols = rng.choice(F, size=n_poisson, replace=False)
    for c in pois_cols:
        col = X[:, c]
        u = special.ndtr(col / col.std())
        u = np.clip(u, 1e-12, 1 - 1e-12)
        X[:, c] = stats.poisson.ppf(u, 4.0)
    _mcar(rng, X, missing)
    block_cols = rng.choice(F, size=n_block, replace=False)
    block_rows = rng.choice(S, size=int(round(block_frac * S)), replace=False)
    if n_block:
        X[np.ix_(block_rows, block_cols)] = np.nan
    return X.astype(np.float32)


def cfg_precision(seed: int = SEED_BASE + 3, S: int = 50_000, F: int = 4_000,
                  missing: float = 0.25) -> np.ndarray:
    rng = _rng(seed)
    mu = rng.uniform(1e3, 1e5, size=F)
    X = factor_matrix(rng, S, F, 5, unit_sd=True)
    X += mu
    _mcar(rng, X, missing)
    return X.astype(np.float32)


@dataclass
class DiffCase:
    X: np.ndarray          # S x F float32 with NaN
    W: np.ndarray          # F x F float64, symmetric
    fd_entries: np.ndarray  # (64, 2) observed (sample, variable) positions
    nan_entries: np.ndarray  # (64, 2) missing positions


def cfg_differentiation(seed: int = SEED_BASE + 4, S: int = 8_192, F: int = 512,
                        missing: float = 0.15, n_fd: int = 64) -> DiffCase:
    rng = _rng(seed)
    X = factor_matrix(rng, S, F, 10)
    _mcar(rng, X, missing)
    W = rng.standard_normal((F, F))
    W = np.triu(W) + np.triu(W, 1).T
    obs = np.argwhere(~np.isnan(X))
    mis = np.argwhere(np.isnan(X))
    fd = obs[rng.choice(len(obs), size=min(n_fd, len(obs)), replace=False)]
    nn = mis[rng.choice(len(mis), size=min(n_fd, len(mis)), replace=False)] if len(mis) else mis
    return DiffCase(X.astype(np.float32), W, fd, nn)


def cfg_serving_base(seed: int = SEED_BASE + 5, S: int = 20_000, F: int = 2_000,
                     missing: float = 0.30) -> np.ndarray:
    rng = _rng(seed)
    X = factor_matrix(rng, S, F, 20)
    _mcar(rng, X, missing)
    return X.astype(np.float32)


@dataclass
class Query:
    arrival_s: float       # arrival time since stream start
    rows: np.ndarray       # int32 sorted sample indices (without replacement)
    cols: np.ndarray       # int32 variable indices (without replacement)
    method: str            # "pearson" or "spearman"


def serving_queries(n: int, S: int, F: int, rate: float = 200.0,
                    seed: int = SEED_BASE + 50, vmin: int = 50, vmax: int = 2_000,
                    fmin: float = 0.1, fmax: float = 0.9) -> list[Query]:
    rng = _rng(seed)
    t = 0.0
    out = []
    vmax = min(vmax, F)
    vmin = min(vmin, vmax)
    for _ in range(n):
        t += rng.exponential(1.0 / rate)
        f = rng.uniform(fmin, fmax)
        nr = max(1, int(round(f * S)))
        rows = np.sort(rng.choice(S, size=nr, replace=False)).astype(np.int32)
        v = int(rng.integers(vmin, vmax + 1))
        cols = rng.choice(F, size=v, replace=False).astype(np.int32)
        method = "pearson" if rng.random() < 0.5 else "spearman"
        out.append(Query(t, rows, cols, method))
    return out


def paper_shape(S: int, F: int, missing: float = 0.10, seed: int = SEED_BASE + 10) -> np.ndarray:
    """Uniform [0,1) values; exactly round(missing*S) missing entries per
    variable at random positions (Section 4.1.1)."""
    rng = _rng(seed)
    X = rng.random((S, F))
    k = int(round(missing * S))
    for c in range(F):
        if k:
            X[rng.choice(S, size=k, replace=False), c] = np.nan
    return X.astype(np.float32)


def heavy_ties(S: int, F: int, levels: int = 5, missing: float = 0.2,
               seed: int = SEED_BASE + 11) -> np.ndarray:
    """Integer-valued columns with few levels (many tied runs), correlated
    through a shared latent factor, with MCAR missingness."""
    rng = _rng(seed)
    base = factor_matrix(rng, S, F, 2)
    X = np.floor((base - base.min()) / (np.ptp(base) + 1e-9) * levels)
    X = np.clip(X, 0, levels - 1)
    _mcar(rng, X, missing)
    return X.astype(np.float32)


def mode_selected(S: int = 2_000, mode_sds=(0.1, 0.01, 0.001), seed: int = SEED_BASE + 15) -> np.ndarray:
    """For each mode sd s: a bimodal column A (modes at -1 and +1, sd s
    around each, half the samples in each), a partner B observed only where A
    is in its upper mode (B = A's deviation there plus independent noise of
    the same size, so r(A, B) is about 0.7), and a partner C observed on
    A's upper mode too but constant there (so C is constant on I(A, C) and
    on I(B, C)); 10% MCAR on top.  Two complete standard normal columns close
    the matrix.  Columns: A_s, B_s, C_s for each s, then the two normals."""
    rng = _rng(seed)
    cols = []
    for sd in mode_sds:
        upper = rng.random(S) < 0.5
        dev = rng.standard_normal(S) * sd
        a = np.where(upper, 1.0, -1.0) + dev
        b = np.where(upper, dev + rng.standard_normal(S) * sd, np.nan)
        c = np.where(upper, 5.0, np.nan)
        for col in (a, b, c):
            col[rng.random(S) < 0.10] = np.nan
            cols.append(col)
    cols.append(rng.standard_normal(S))
    cols.append(rng.standard_normal(S))
    return np.column_stack(cols).astype(np.float32)


def edge_matrix() -> np.ndarray:
    """Hand-built 8 x 10 matrix whose column pairs cover the degenerate cases:
    0, 1, 2 and 3 pairwise-complete samples, a column constant on its observed
    entries, an all-missing column, a column constant on a pair subset,
    all-tied and partly tied columns and an exact linear relation.
    """
    n = math.nan
    cols = [
        [1.0, 2.0, 3.0, 4.0, 5.0, 6.0, 7.0, 8.0],      # 0 full, increasing
        [2.0, 4.0, 6.0, 8.0, 10.0, 12.0, 14.0, 16.0],  # 1 exact linear of 0
        [n, n, n, n, n, n, n, n],                      # 2 all missing
        [3.0, 3.0, 3.0, 3.0, 3.0, 3.0, 3.0, 3.0],      # 3 constant
        [5.0, n, n, n, n, n, n, n],                    # 4 one observed
        [1.0, 7.0, n, n, n, n, n, n],                  # 5 two observed
        [9.0, 1.0, 4.0, n, n, n, n, n],                # 6 three observed
        [1.0, 1.0, 2.0, 2.0, 2.0, 3.0, 1.0, 2.0],      # 7 heavy ties
        [4.0, 4.0, 4.0, 4.0, 1.0, 2.0, 3.0, 5.0],      # 8 constant on rows 0-3
        [-0.0, 0.0, 1.0, -1.0, n, 2.0, -0.0, 0.5],     # 9 signed zeros tie
    ]
    return np.array(cols, dtype=np.float32).T.copy()


def pvalue_matrix(F: int, seed: int = SEED_BASE + 12, nan_frac: float = 0.02,
                  tie_frac: float = 0.2) -> np.ndarray:
    """Symmetric F x F float64 matrix of p-values for the multiple-testing
    correction: 30% log-uniform on [1e-12, 1] (strong associations), the rest
    uniform on [0, 1) (null pairs); a tie_frac share rounded to 2 decimals
    (groups of equal values); the first two pairs exactly 0 and 1; a nan_frac
    share undefined (NaN).  The diagonal holds 0.5 (it is not a test)."""
    rng = _rng(seed)
    n = F * (F - 1) // 2
    v = np.where(rng.random(n) < 0.3, 10.0 ** -rng.uniform(0, 12, n), rng.random(n))
    tie = rng.random(n) < tie_frac
    v[tie] = np.round(v[tie], 2)
    if n > 4:
        v[0] = 0.0
        v[1] = 1.0
    v[rng.random(n) < nan_frac] = np.nan
    P = np.full((F, F), 0.5)
    iu, ju = np.triu_indices(F, 1)
    P[iu, ju] = v
    P[ju, iu] = v
    return P


def categorical_continuous(S: int, FC: int, FQ: int, ncat: int, missing: float = 0.3,
                           seed: int = SEED_BASE + 13):
    """Label-encoded categorical features (labels 0 .. ncat-1, every label
    present in every column, as in the paper's simulated categorical data) and
    continuous features; a third of the continuous columns are shifted by
    0.3 sd per label of a random categorical column (so that some pairs carry
    an effect); MCAR missingness at `missing` on both matrices.  Returns
    (L, X) float32, samples x features."""
    rng = _rng(seed)
    L = rng.integers(0, ncat, size=(S, FC)).astype(np.float64)
    if S >= ncat:
        L[:ncat, :] = np.arange(ncat)[:, None]
    X = rng.normal(size=(S, FQ)) * rng.uniform(0.5, 3.0, FQ) + rng.uniform(-50.0, 50.0, FQ)
    src = rng.integers(0, FC, size=FQ)
    eff = rng.random(FQ) < 1.0 / 3.0
    X[:, eff] += 0.3 * L[:, src[eff]]
    _mcar(rng, L, missing)
    _mcar(rng, X, missing)
    return L.astype(np.float32), X.astype(np.float32)


def categorical_matrix(S: int, F: int, ncat: int, missing: float = 0.3, seed: int = SEED_BASE + 14) -> np.ndarray:
    """Label-encoded categorical features (labels 0 .. c_j - 1 with c_j drawn
    from 2 .. ncat per column, every label present): quantiles of a rank-3
    factor model, so that columns sharing factors are dependent; MCAR
    missingness.  Returns S x F float32."""
    rng = _rng(seed)
    Z = factor_matrix(rng, S, F, 3)
    L = np.empty((S, F))
    for j in range(F):
        c = int(rng.integers(2, ncat + 1))
        edges = np.quantile(Z[:, j], np.linspace(0, 1, c + 1)[1:-1])
        L[:, j] = np.searchsorted(edges, Z[:, j])
        if S >= c:
            L[:c, j] = np.arange(c)
    _mcar(rng, L, missing)
    return L.astype(np.float32)
