"""ctypes binding of libnapy.so: argument marshalling only.

Every function of include/napy.h is bound here under the same name.  The
library must be built (``python -m paper_2505_00448_amd.build``); loading fails
loudly otherwise -- there is no fallback implementation.
"""

from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libnapy.so")

NAPY_OK = 0
NAPY_E_INVALID = 1
NAPY_E_WORKSPACE = 2
NAPY_E_UNSUPPORTED = 3
NAPY_E_HIP = 4

PREC = {"fp32": 0, "bf16x3": 1, "fp64": 2}

# Every symbol declared in include/napy.h.
EXPORTS = [
    "napy_strerror", "napy_last_error", "napy_version",
    "napy_pearson_workspace", "napy_pearson", "napy_pearson_noalloc",
    "napy_spearman_workspace", "napy_spearman",
    "napy_pearson_profiled", "napy_spearman_profiled",
    "napy_pearson_fwd", "napy_pearson_backward_workspace", "napy_pearson_backward",
    "napy_pearson_subset_workspace", "napy_pearson_subset",
    "napy_spearman_base_bytes", "napy_spearman_base_prepare",
    "napy_spearman_subset_workspace", "napy_spearman_subset",
    "napy_spearman_pair_ranks", "napy_pvalue_device", "napy_pvalue_host",
    "napy_adjust_workspace", "napy_adjust_pvalues",
    "napy_ttest_workspace", "napy_ttest", "napy_anova_workspace", "napy_anova", "napy_fdist_sf_host",
    "napy_chi2_workspace", "napy_chi2", "napy_chi2_sf_host",
    "napy_mannwhitney_workspace", "napy_mannwhitney", "napy_kruskal_workspace", "napy_kruskal",
]


class NapyOpts(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("use_sentinel", ctypes.c_int32),
                ("sentinel", ctypes.c_float), ("reserved", ctypes.c_int32)]


class NapyError(RuntimeError):
    def __init__(self, status: int, what: str):
        self.status = status
        super().__init__(what)


_lib = None


def load() -> ctypes.CDLL:
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is missing: build it with `python -m paper_2505_00448_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    i64 = ctypes.c_int64
    i32 = ctypes.c_int32
    sz = ctypes.c_size_t
    O = ctypes.POINTER(NapyOpts)
    sig = {
        "napy_strerror": (ctypes.c_char_p, [ctypes.c_int]),
        "napy_last_error": (ctypes.c_char_p, []),
        "napy_version": (ctypes.c_char_p, []),
        "napy_pearson_workspace": (sz, [i64, i64, O]),
        "napy_pearson": (ctypes.c_int, [P, i64, i64, i64, P, P, P, i64, P, sz, O, P]),
        "napy_pearson_noalloc": (ctypes.c_int, [P, i64, i64, i64, P, P, P, i64, O, P]),
        "napy_spearman_workspace": (sz, [i64, i64, O]),
        "napy_spearman": (ctypes.c_int, [P, i64, i64, i64, P, P, P, i64, P, sz, O, P]),
        "napy_pearson_profiled": (ctypes.c_int, [P, i64, i64, i64, P, P, P, i64, P, sz, O, P, P]),
        "napy_spearman_profiled": (ctypes.c_int, [P, i64, i64, i64, P, P, P, i64, P, sz, O, P, P]),
        "napy_pearson_fwd": (ctypes.c_int, [P, i64, i64, i64, P, P, P, i64, P, P, sz, O, P]),
        "napy_pearson_backward_workspace": (sz, [i64, i64, O]),
        "napy_pearson_backward": (ctypes.c_int, [P, i64, i64, i64, P, P, i64, P, i64, P, sz, O, P]),
        "napy_pearson_subset_workspace": (sz, [i64, i64, O]),
        "napy_pearson_subset": (ctypes.c_int, [P, i64, i64, i64, P, i64, P, i64, P, P, P, i64, P, sz, O, P]),
        "napy_spearman_base_bytes": (sz, [i64, i64]),
        "napy_spearman_base_prepare": (ctypes.c_int, [P, i64, i64, i64, P, sz, O, P]),
        "napy_spearman_subset_workspace": (sz, [i64, i64, i64, O]),
        "napy_spearman_subset": (ctypes.c_int, [P, i64, i64, P, i64, P, i64, P, P, P, i64, P, sz, O, P]),
        "napy_spearman_pair_ranks": (ctypes.c_int, [P, i64, i64, i64, i32, i32, P, P, P, sz, O, P]),
        "napy_pvalue_device": (ctypes.c_int, [P, P, P, i64, P]),
        "napy_pvalue_host": (ctypes.c_int, [P, P, P, i64]),
        "napy_adjust_workspace": (sz, [i64]),
        "napy_adjust_pvalues": (ctypes.c_int, [P, i64, i64, P, i64, i32, P, sz, P]),
        "napy_ttest_workspace": (sz, [i64, i64, i64, O]),
        "napy_ttest": (ctypes.c_int, [P, i64, P, i64, i64, i64, i64, i32, P, P, P, i64, P, sz, O, P]),
        "napy_anova_workspace": (sz, [i64, i64, i64, i32, O]),
        "napy_anova": (ctypes.c_int, [P, i64, P, i64, i64, i64, i64, i32, P, P, P, i64, P, sz, O, P]),
        "napy_fdist_sf_host": (ctypes.c_int, [P, P, P, P, i64]),
        "napy_chi2_workspace": (sz, [i64, i64, i32, O]),
        "napy_chi2": (ctypes.c_int, [P, i64, i64, i64, i32, P, P, P, P, i64, P, sz, O, P]),
        "napy_chi2_sf_host": (ctypes.c_int, [P, P, P, i64]),
        "napy_mannwhitney_workspace": (sz, [i64, i64, i64, O]),
        "napy_mannwhitney": (ctypes.c_int, [P, i64, P, i64, i64, i64, i64, i32, P, P, P, i64, P, sz, O, P]),
        "napy_kruskal_workspace": (sz, [i64, i64, i64, i32, O]),
        "napy_kruskal": (ctypes.c_int, [P, i64, P, i64, i64, i64, i64, i32, P, P, P, i64, P, sz, O, P]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def make_opts(precision: str = "fp32", missing=None) -> NapyOpts:
    import math
    o = NapyOpts()
    o.precision = PREC[precision]
    if missing is None or (isinstance(missing, float) and math.isnan(missing)):
        o.use_sentinel = 0
        o.sentinel = 0.0
    else:
        o.use_sentinel = 1
        o.sentinel = float(missing)
    o.reserved = 0
    return o


def check(status: int, what: str) -> None:
    if status != NAPY_OK:
        lib = load()
        msg = lib.napy_strerror(status).decode()
        detail = lib.napy_last_error().decode()
        raise NapyError(status, f"{what}: {msg}" + (f" ({detail})" if detail else ""))
