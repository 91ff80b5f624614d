"""PyTorch-facing wrappers of libnapy (device memory and streams only; every
step of the computation runs in the HIP kernels behind the C ABI).

Outputs follow the paper's convention of a dict of F x F matrices
(NApy, Section 3.4): "r" (Pearson r or Spearman rho, float64), "p" (two-sided
p-value, float64) and "n" (pairwise-complete sample count, int32).
"""

from __future__ import annotations

import ctypes
from typing import Iterable, Optional

import torch

from . import _lib

_OUT_KEYS = ("r", "p", "n")


def _ptr(t: Optional[torch.Tensor]):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _stream_handle(device: torch.device) -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _prep_input(X: torch.Tensor, samples_axis: int, check_finite: bool) -> torch.Tensor:
    if not isinstance(X, torch.Tensor) or X.dim() != 2:
        raise TypeError("X must be a 2-D torch tensor")
    if not X.is_cuda:
        raise ValueError("X must be a CUDA (ROCm) tensor on the MI355X")
    if samples_axis == 1:
        X = X.t()
    elif samples_axis != 0:
        raise ValueError("samples_axis must be 0 (rows are samples) or 1 (rows are variables)")
    if X.dtype != torch.float32:
        X = X.to(torch.float32)
    if X.stride(1) != 1 or X.stride(0) < X.shape[1]:
        X = X.contiguous()
    if X.shape[0] == 0 and X.stride(0) < X.shape[1]:
        X = torch.empty((0, X.shape[1]), dtype=torch.float32, device=X.device)
    if check_finite and bool(torch.isinf(X).any()):
        raise ValueError("X contains +-Inf; only NaN (or the chosen sentinel) may mark missing values")
    return X


def _outputs(F: int, device, outputs: Iterable[str]):
    want = set(outputs)
    bad = want - set(_OUT_KEYS)
    if bad:
        raise ValueError(f"unknown outputs {sorted(bad)}; choose from {_OUT_KEYS}")
    r = torch.empty((F, F), dtype=torch.float64, device=device) if "r" in want else None
    p = torch.empty((F, F), dtype=torch.float64, device=device) if "p" in want else None
    n = torch.empty((F, F), dtype=torch.int32, device=device) if "n" in want else None
    return r, p, n


def _workspace(nbytes: int, device) -> torch.Tensor:
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)


def pearson(X: torch.Tensor, precision: str = "fp32", missing: Optional[float] = None,
            outputs: Iterable[str] = _OUT_KEYS, samples_axis: int = 0,
            check_finite: bool = True, workspace: Optional[torch.Tensor] = None) -> dict:
    """All-pairs Pearson with pairwise deletion.  precision: "fp32",
    "bf16x3" or "fp64" (validation)."""
    lib = _lib.load()
    X = _prep_input(X, samples_axis, check_finite)
    S, F = X.shape
    opts = _lib.make_opts(precision, missing)
    need = lib.napy_pearson_workspace(S, F, ctypes.byref(opts))
    if need == 0:
        raise _lib.NapyError(_lib.NAPY_E_UNSUPPORTED, f"napy_pearson_workspace({S}, {F}) refused the shape")
    ws = workspace if workspace is not None and workspace.numel() >= need else _workspace(need, X.device)
    r, p, n = _outputs(F, X.device, outputs)
    st = lib.napy_pearson(_ptr(X), S, F, X.stride(0), _ptr(r), _ptr(p), _ptr(n), F,
                          _ptr(ws), ws.numel(), ctypes.byref(opts), _stream_handle(X.device))
    _lib.check(st, "napy_pearson")
    return {k: v for k, v in zip(_OUT_KEYS, (r, p, n)) if v is not None}


def spearman(X: torch.Tensor, missing: Optional[float] = None,
             outputs: Iterable[str] = _OUT_KEYS, samples_axis: int = 0,
             check_finite: bool = True, workspace: Optional[torch.Tensor] = None) -> dict:
    """All-pairs Spearman with pairwise deletion (average ranks for ties)."""
    lib = _lib.load()
    X = _prep_input(X, samples_axis, check_finite)
    S, F = X.shape
    opts = _lib.make_opts("fp32", missing)
    need = lib.napy_spearman_workspace(S, F, ctypes.byref(opts))
    if need == 0:
        raise _lib.NapyError(_lib.NAPY_E_UNSUPPORTED, f"napy_spearman_workspace({S}, {F}) refused the shape")
    ws = workspace if workspace is not None and workspace.numel() >= need else _workspace(need, X.device)
    r, p, n = _outputs(F, X.device, outputs)
    st = lib.napy_spearman(_ptr(X), S, F, X.stride(0), _ptr(r), _ptr(p), _ptr(n), F,
                           _ptr(ws), ws.numel(), ctypes.byref(opts), _stream_handle(X.device))
    _lib.check(st, "napy_spearman")
    return {k: v for k, v in zip(_OUT_KEYS, (r, p, n)) if v is not None}


def spearman_pair_ranks(X: torch.Tensor, g: int, h: int, missing: Optional[float] = None):
    """Test hook: doubled average ranks inside I(g,h) in sample order (-1 for
    samples outside I(g,h)) as assigned by the GPU path."""
    lib = _lib.load()
    X = _prep_input(X, 0, False)
    S, F = X.shape
    opts = _lib.make_opts("fp32", missing)
    need = lib.napy_spearman_workspace(S, F, ctypes.byref(opts))
    ws = _workspace(need, X.device)
    rg = torch.empty(max(S, 1), dtype=torch.int32, device=X.device)
    rh = torch.empty(max(S, 1), dtype=torch.int32, device=X.device)
    st = lib.napy_spearman_pair_ranks(_ptr(X), S, F, X.stride(0), int(g), int(h), _ptr(rg), _ptr(rh),
                                      _ptr(ws), ws.numel(), ctypes.byref(opts), _stream_handle(X.device))
    _lib.check(st, "napy_spearman_pair_ranks")
    return rg[:S], rh[:S]


def _groups_call(kind: str, L: torch.Tensor, X: torch.Tensor, welch: bool, ncat: Optional[int],
                 missing: Optional[float], samples_axis: int, workspace: Optional[torch.Tensor]) -> dict:
    lib = _lib.load()
    L = _prep_input(L, samples_axis, False)
    X = _prep_input(X, samples_axis, True)
    if L.shape[0] != X.shape[0] or L.device != X.device:
        raise ValueError("L and X must have the same samples on the same device")
    S, FC = L.shape
    FQ = X.shape[1]
    opts = _lib.make_opts("fp64", missing)
    if kind in ("anova", "kruskal") and ncat is None:
        # largest observed label + 1 (one device reduction)
        lab = L if missing is None else torch.where(L == missing, torch.nan, L)
        mx = torch.nan_to_num(lab, nan=-1.0).max() if L.numel() else torch.tensor(-1.0)
        ncat = max(2, int(mx.item()) + 1)
    if kind == "ttest":
        need = lib.napy_ttest_workspace(S, FC, FQ, ctypes.byref(opts))
    elif kind == "anova":
        need = lib.napy_anova_workspace(S, FC, FQ, int(ncat), ctypes.byref(opts))
    elif kind == "mannwhitney":
        need = lib.napy_mannwhitney_workspace(S, FC, FQ, ctypes.byref(opts))
    else:
        need = lib.napy_kruskal_workspace(S, FC, FQ, int(ncat), ctypes.byref(opts))
    if need == 0:
        raise _lib.NapyError(_lib.NAPY_E_UNSUPPORTED, f"{kind} workspace refused S={S} FC={FC} FQ={FQ}")
    ws = workspace if workspace is not None and workspace.numel() >= need else _workspace(need, X.device)
    stat = torch.empty((FC, FQ), dtype=torch.float64, device=X.device)
    p = torch.empty((FC, FQ), dtype=torch.float64, device=X.device)
    n = torch.empty((FC, FQ), dtype=torch.int32, device=X.device)
    args = (_ptr(L), L.stride(0), _ptr(X), X.stride(0), S, FC, FQ)
    tail = (_ptr(stat), _ptr(p), _ptr(n), FQ, _ptr(ws), ws.numel(), ctypes.byref(opts), _stream_handle(X.device))
    if kind == "ttest":
        _lib.check(lib.napy_ttest(*args, int(bool(welch)), *tail), "napy_ttest")
        return {"t": stat, "p": p, "n": n}
    if kind == "anova":
        _lib.check(lib.napy_anova(*args, int(ncat), *tail), "napy_anova")
        return {"F": stat, "p": p, "n": n}
    if kind == "mannwhitney":
        _lib.check(lib.napy_mannwhitney(*args, int(welch), *tail), "napy_mannwhitney")
        return {"U": stat, "p": p, "n": n}
    _lib.check(lib.napy_kruskal(*args, int(ncat), *tail), "napy_kruskal")
    return {"H": stat, "p": p, "n": n}


def ttest(L: torch.Tensor, X: torch.Tensor, welch: bool = False, missing: Optional[float] = None,
          samples_axis: int = 0, workspace: Optional[torch.Tensor] = None) -> dict:
    """Two-sample t-tests of every dichotomous column of L (labels 0/1)
    against every continuous column of X with pairwise deletion (NApy,
    Section 3.5): {"t", "p", "n"}, FC x FQ.  welch=False: Student."""
    return _groups_call("ttest", L, X, welch, None, missing, samples_axis, workspace)


def anova(L: torch.Tensor, X: torch.Tensor, ncat: Optional[int] = None, missing: Optional[float] = None,
          samples_axis: int = 0, workspace: Optional[torch.Tensor] = None) -> dict:
    """One-way ANOVA of every categorical column of L (labels 0 .. ncat-1)
    against every continuous column of X with pairwise deletion (NApy,
    Section 3.5): {"F", "p", "n"}, FC x FQ.  ncat defaults to the largest
    observed label + 1."""
    return _groups_call("anova", L, X, False, ncat, missing, samples_axis, workspace)


_MWU_MODE = {"auto": 0, "asymptotic": 1}


def mannwhitney(L: torch.Tensor, X: torch.Tensor, mode: str = "auto", missing: Optional[float] = None,
                samples_axis: int = 0, workspace: Optional[torch.Tensor] = None) -> dict:
    """Mann-Whitney U tests of every dichotomous column of L (labels 0/1)
    against every continuous column of X with pairwise deletion (NApy,
    Section 3.5): {"U" (of label 0), "p", "n"}, FC x FQ.  mode "auto": exact
    p when the pair has no ties and a group has fewer than eight samples,
    else asymptotic; "asymptotic": always the normal approximation."""
    if mode not in _MWU_MODE:
        raise ValueError(f"mode must be one of {sorted(_MWU_MODE)}")
    return _groups_call("mannwhitney", L, X, _MWU_MODE[mode], None, missing, samples_axis, workspace)


def kruskal(L: torch.Tensor, X: torch.Tensor, ncat: Optional[int] = None, missing: Optional[float] = None,
            samples_axis: int = 0, workspace: Optional[torch.Tensor] = None) -> dict:
    """Kruskal-Wallis H tests of every categorical column of L (labels 0 ..
    ncat-1) against every continuous column of X with pairwise deletion
    (NApy, Section 3.5): {"H", "p", "n"}, FC x FQ.  ncat defaults to the
    largest observed label + 1."""
    return _groups_call("kruskal", L, X, False, ncat, missing, samples_axis, workspace)


def chi2(L: torch.Tensor, ncat: Optional[int] = None, missing: Optional[float] = None, samples_axis: int = 0,
         workspace: Optional[torch.Tensor] = None) -> dict:
    """Chi-squared tests of independence of every pair of label-encoded
    categorical columns of L with pairwise deletion (NApy, Section 3.5):
    {"chi2", "p", "v" (Cramer's V), "n"}, F x F.  ncat defaults to the
    largest observed label + 1."""
    lib = _lib.load()
    L = _prep_input(L, samples_axis, False)
    S, F = L.shape
    opts = _lib.make_opts("fp64", missing)
    if ncat is None:
        lab = L if missing is None else torch.where(L == missing, torch.nan, L)
        mx = torch.nan_to_num(lab, nan=-1.0).max() if L.numel() else torch.tensor(-1.0)
        ncat = max(2, int(mx.item()) + 1)
    need = lib.napy_chi2_workspace(S, F, int(ncat), ctypes.byref(opts))
    if need == 0:
        raise _lib.NapyError(_lib.NAPY_E_UNSUPPORTED, f"chi2 workspace refused S={S} F={F} ncat={ncat}")
    ws = workspace if workspace is not None and workspace.numel() >= need else _workspace(need, L.device)
    out = {k: torch.empty((F, F), dtype=torch.float64, device=L.device) for k in ("chi2", "p", "v")}
    out["n"] = torch.empty((F, F), dtype=torch.int32, device=L.device)
    st = lib.napy_chi2(_ptr(L), L.stride(0), S, F, int(ncat), _ptr(out["chi2"]), _ptr(out["p"]), _ptr(out["v"]),
                       _ptr(out["n"]), F, _ptr(ws), ws.numel(), ctypes.byref(opts), _stream_handle(L.device))
    _lib.check(st, "napy_chi2")
    return out


_ADJUST = {"bonferroni": 0, "bh": 1, "by": 2}


def adjust_pvalues(P: torch.Tensor, method: str = "bh", out: Optional[torch.Tensor] = None,
                   workspace: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Multiple-testing correction of a symmetric F x F p matrix (NApy,
    Section 3.4): "bonferroni", "bh" (Benjamini-Hochberg) or "by"
    (Benjamini-Yekutieli).  The tests are the pairs i < j with a defined p;
    the diagonal and undefined pairs are NaN in the result.  ``out`` may be
    ``P`` itself (in-place)."""
    if method not in _ADJUST:
        raise ValueError(f"method must be one of {sorted(_ADJUST)}")
    if not isinstance(P, torch.Tensor) or P.dim() != 2 or P.shape[0] != P.shape[1]:
        raise TypeError("P must be a square 2-D torch tensor")
    if not P.is_cuda:
        raise ValueError("P must be a CUDA (ROCm) tensor on the MI355X")
    lib = _lib.load()
    if P.dtype != torch.float64 or P.stride(1) != 1:
        P = P.to(torch.float64).contiguous()
    F = P.shape[0]
    if out is None:
        out = torch.empty((F, F), dtype=torch.float64, device=P.device)
    elif out.shape != P.shape or out.dtype != torch.float64 or out.stride(1) != 1 or out.device != P.device:
        raise ValueError("out must be a float64 F x F row-major tensor on P's device")
    need = lib.napy_adjust_workspace(F)
    if need == 0:
        raise _lib.NapyError(_lib.NAPY_E_UNSUPPORTED, f"napy_adjust_workspace({F}) refused the shape")
    ws = workspace if workspace is not None and workspace.numel() >= need else _workspace(need, P.device)
    st = lib.napy_adjust_pvalues(_ptr(P), F, P.stride(0), _ptr(out), out.stride(0), _ADJUST[method],
                                 _ptr(ws), ws.numel(), _stream_handle(P.device))
    _lib.check(st, "napy_adjust_pvalues")
    return out


def pvalue_device(r: torch.Tensor, n: torch.Tensor) -> torch.Tensor:
    """Test hook: the library's device p-value routine on (r, n) arrays."""
    lib = _lib.load()
    r = r.to(torch.float64).contiguous()
    n = n.to(torch.int32).contiguous()
    p = torch.empty_like(r)
    st = lib.napy_pvalue_device(_ptr(r), _ptr(n), _ptr(p), r.numel(), _stream_handle(r.device))
    _lib.check(st, "napy_pvalue_device")
    return p


# ---------------------------------------------------------------------------
# differentiation
# ---------------------------------------------------------------------------

class PearsonCorr(torch.autograd.Function):
    """R = pairwise-deletion Pearson matrix of X (samples x variables) with a
    hand-written backward (libnapy's napy_pearson_backward).  R is float64;
    undefined entries are NaN in the forward and pass no gradient."""

    @staticmethod
    def forward(ctx, X: torch.Tensor, precision: str = "fp32"):
        lib = _lib.load()
        Xc = _prep_input(X.detach(), 0, True)
        S, F = Xc.shape
        opts = _lib.make_opts(precision)
        need = lib.napy_pearson_workspace(S, F, ctypes.byref(opts))
        ws = _workspace(need, Xc.device)
        r = torch.empty((F, F), dtype=torch.float64, device=Xc.device)
        saved = torch.empty((7, F, F), dtype=torch.float64, device=Xc.device)
        st = lib.napy_pearson_fwd(_ptr(Xc), S, F, Xc.stride(0), _ptr(r), None, None, F, _ptr(saved),
                                  _ptr(ws), ws.numel(), ctypes.byref(opts), _stream_handle(Xc.device))
        _lib.check(st, "napy_pearson_fwd")
        ctx.save_for_backward(Xc, saved)
        ctx.precision = precision
        ctx.in_dtype = X.dtype
        return r

    @staticmethod
    def backward(ctx, dR: torch.Tensor):
        lib = _lib.load()
        Xc, saved = ctx.saved_tensors
        S, F = Xc.shape
        opts = _lib.make_opts(ctx.precision)
        dRf = torch.nan_to_num(dR.detach().to(torch.float32)).contiguous()
        need = lib.napy_pearson_backward_workspace(S, F, ctypes.byref(opts))
        ws = _workspace(need, Xc.device)
        dX = torch.empty((S, F), dtype=torch.float32, device=Xc.device)
        st = lib.napy_pearson_backward(_ptr(Xc), S, F, Xc.stride(0), _ptr(saved), _ptr(dRf), F, _ptr(dX), F,
                                       _ptr(ws), ws.numel(), ctypes.byref(opts), _stream_handle(Xc.device))
        _lib.check(st, "napy_pearson_backward")
        return dX.to(ctx.in_dtype), None


def pearson_corr(X: torch.Tensor, precision: str = "fp32") -> torch.Tensor:
    return PearsonCorr.apply(X, precision)


# ---------------------------------------------------------------------------
# subset queries on a resident base
# ---------------------------------------------------------------------------

def pearson_subset(X: torch.Tensor, rows: torch.Tensor, cols: torch.Tensor, precision: str = "fp32",
                   missing: Optional[float] = None, stream=None, workspace=None, out=None) -> dict:
    lib = _lib.load()
    S, F = X.shape
    Sq, Fq = int(rows.numel()), int(cols.numel())
    opts = _lib.make_opts(precision, missing)
    need = lib.napy_pearson_subset_workspace(Sq, Fq, ctypes.byref(opts))
    ws = workspace if workspace is not None and workspace.numel() >= need else _workspace(need, X.device)
    r, p, n = out if out is not None else _outputs(Fq, X.device, _OUT_KEYS)
    sh = ctypes.c_void_p(stream.cuda_stream) if stream is not None else _stream_handle(X.device)
    st = lib.napy_pearson_subset(_ptr(X), S, F, X.stride(0), _ptr(rows), Sq, _ptr(cols), Fq,
                                 _ptr(r), _ptr(p), _ptr(n), Fq, _ptr(ws), ws.numel(), ctypes.byref(opts), sh)
    _lib.check(st, "napy_pearson_subset")
    return {"r": r, "p": p, "n": n}


class SpearmanBase:
    """A base matrix whose columns are sorted once (resident on the device);
    Spearman subset queries then only compact those sorted orders."""

    def __init__(self, X: torch.Tensor, missing: Optional[float] = None):
        lib = _lib.load()
        X = _prep_input(X, 0, True)
        self.S, self.F = X.shape
        self.missing = missing
        opts = _lib.make_opts("fp32", missing)
        nbytes = lib.napy_spearman_base_bytes(self.S, self.F)
        if nbytes == 0:
            raise _lib.NapyError(_lib.NAPY_E_UNSUPPORTED, "napy_spearman_base_bytes refused the shape")
        self.buf = _workspace(nbytes, X.device)
        st = lib.napy_spearman_base_prepare(_ptr(X), self.S, self.F, X.stride(0), _ptr(self.buf),
                                            self.buf.numel(), ctypes.byref(opts), _stream_handle(X.device))
        _lib.check(st, "napy_spearman_base_prepare")

    def subset(self, rows: torch.Tensor, cols: torch.Tensor, stream=None, workspace=None, out=None) -> dict:
        lib = _lib.load()
        Sq, Fq = int(rows.numel()), int(cols.numel())
        opts = _lib.make_opts("fp32", self.missing)
        need = lib.napy_spearman_subset_workspace(self.S, Sq, Fq, ctypes.byref(opts))
        dev = self.buf.device
        ws = workspace if workspace is not None and workspace.numel() >= need else _workspace(need, dev)
        r, p, n = out if out is not None else _outputs(Fq, dev, _OUT_KEYS)
        sh = ctypes.c_void_p(stream.cuda_stream) if stream is not None else _stream_handle(dev)
        st = lib.napy_spearman_subset(_ptr(self.buf), self.S, self.F, _ptr(rows), Sq, _ptr(cols), Fq,
                                      _ptr(r), _ptr(p), _ptr(n), Fq, _ptr(ws), ws.numel(),
                                      ctypes.byref(opts), sh)
        _lib.check(st, "napy_spearman_subset")
        return {"r": r, "p": p, "n": n}
