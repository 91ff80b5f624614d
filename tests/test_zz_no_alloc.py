"""GPU test of napy_pearson_noalloc, the allocation-free Pearson entry point
(its workspace is the library's fixed per-device scratch array): through the
C ABI, two calls in a row -- the second on a smaller input, so it runs over
the first call's leftover scratch contents -- each checked against
napy_pearson on the same input to the parity bars (counts exact, r within
1e-6, NaN placement exact, p through its conditioning); and a shape whose
scratch need exceeds the array is refused on the host with
NAPY_E_UNSUPPORTED."""

import ctypes

import numpy as np
import pytest

import synth
from parity_util import assert_counts_equal, assert_p_close, assert_r_close

pytestmark = pytest.mark.gpu


def _call_pair(lib, _lib, X, dev, precision):
    import torch
    Xd = torch.from_numpy(np.ascontiguousarray(X, dtype=np.float32)).to(dev)
    S, F = X.shape
    o = _lib.make_opts(precision)
    P = lambda t: ctypes.c_void_p(t.data_ptr())
    sh = ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)
    outs = []
    for noalloc in (False, True):
        r = torch.full((F, F), 7.0, dtype=torch.float64, device=dev)
        p = torch.full((F, F), 7.0, dtype=torch.float64, device=dev)
        n = torch.full((F, F), -7, dtype=torch.int32, device=dev)
        if noalloc:
            st = lib.napy_pearson_noalloc(P(Xd), S, F, F, P(r), P(p), P(n), F, ctypes.byref(o), sh)
        else:
            need = lib.napy_pearson_workspace(S, F, ctypes.byref(o))
            ws = torch.empty(need, dtype=torch.uint8, device=dev)
            st = lib.napy_pearson(P(Xd), S, F, F, P(r), P(p), P(n), F, P(ws), need, ctypes.byref(o), sh)
        _lib.check(st, "noalloc" if noalloc else "napy_pearson")
        torch.cuda.synchronize(dev)
        outs.append((r.cpu().numpy(), p.cpu().numpy(), n.cpu().numpy()))
    return outs


@pytest.mark.parametrize("precision", ["bf16x3", "fp32"])
def test_noalloc_matches_napy_pearson(gpu_device, precision):
    from paper_2505_00448_amd import _lib
    lib = _lib.load()
    big = synth.cfg_gpu_headline(S=6000, F=700)
    small = synth.mode_selected(S=900)
    for where, X in (("first call, 6000 x 700", big), ("second call, 900 x 11", small)):
        print(f"[noalloc] {precision} {where}", flush=True)
        (r0, p0, n0), (r1, p1, n1) = _call_pair(lib, _lib, X, gpu_device, precision)
        assert_counts_equal(n1, n0, where)
        worst = assert_r_close(r1, r0, 1e-6, where)
        assert_p_close(p1, p0, r0, n0, max(worst, 1e-15), where)
        assert np.array_equal(r1, r1.T, equal_nan=True)


def test_noalloc_refuses_oversized(gpu_device):
    from paper_2505_00448_amd import _lib
    lib = _lib.load()
    o = _lib.make_opts("bf16x3")
    F = 4000  # split-K partials of 8,000 tiles alone exceed the 128 MiB array
    fake = ctypes.c_void_p(0x1000)  # refused on the host before any device access
    st = lib.napy_pearson_noalloc(fake, 1000, F, F, fake, fake, fake, F, ctypes.byref(o), None)
    assert st == _lib.NAPY_E_UNSUPPORTED
    assert b"128" in lib.napy_last_error() or b"scratch" in lib.napy_last_error()
