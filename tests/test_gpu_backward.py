"""GPU parity of the masked-Pearson backward (napy_pearson_backward behind
torch.autograd): against the FP64 CPU autograd reference of the oracle and
against central finite differences of the FP64 loss.

Bars: max |dX - ref| <= 1e-4 * max |ref| (FP32 GEMMs, FP64 coefficients);
FD: relative 1e-2 at h = 1e-3; missing entries exactly 0.
"""

import numpy as np
import pytest

import synth
from oracle import grad as ograd

pytestmark = pytest.mark.gpu


def _row_r(X, c):
    """r_{c,h} for all h in FP64 from the two-pass definition (vectorised
    over h): used for finite differences of the loss in one column."""
    M = ~np.isnan(X)
    X0 = np.where(M, X, 0.0)
    m = M[:, c:c + 1] & M
    n = m.sum(0).astype(np.float64)
    xc = np.where(m, X0[:, c:c + 1], 0.0)
    xh = np.where(m, X0, 0.0)
    with np.errstate(invalid="ignore", divide="ignore"):
        mc = xc.sum(0) / n
        mh = xh.sum(0) / n
        dc = np.where(m, xc - mc, 0.0)
        dh = np.where(m, xh - mh, 0.0)
        r = (dc * dh).sum(0) / np.sqrt((dc * dc).sum(0) * (dh * dh).sum(0))
    r[c] = 0.0
    return np.nan_to_num(r)


def _gpu_grad(X, W, dev, precision):
    import torch
    import paper_2505_00448_amd as napy
    Xt = torch.from_numpy(X).to(dev).requires_grad_(True)
    R = napy.pearson_corr(Xt, precision)
    Wt = torch.from_numpy(W).to(dev)
    loss = (torch.nan_to_num(R) * Wt).sum()
    loss.backward()
    return Xt.grad.detach().cpu().numpy().astype(np.float64)


@pytest.mark.parametrize("precision", ["fp32", "bf16x3", "fp64"])
def test_backward_small(gpu_device, precision):
    case = synth.cfg_differentiation(S=700, F=70, n_fd=16)
    X = case.X
    W = case.W[:70, :70]
    _, ref, _ = ograd.pearson_loss_grad(X.astype(np.float64), W)
    g = _gpu_grad(X, W, gpu_device, precision)
    miss = np.isnan(X)
    assert np.all(g[miss] == 0.0)
    err = np.abs(g - ref).max() / np.abs(ref).max()
    assert err <= 1e-4, err


def test_backward_mode_selected(gpu_device):
    """Pairs whose complete samples sit 10 and 100 of their own sds from the
    column mean (the forward recomputes them in FP64, and the backward takes
    their saved sums and r from there), and partners constant on the pair
    (undefined r: no gradient)."""
    X = synth.mode_selected(S=900, mode_sds=(0.1, 0.01))
    F = X.shape[1]
    rng = np.random.default_rng(5)
    W = rng.standard_normal((F, F))
    W = np.triu(W) + np.triu(W, 1).T
    _, ref, _ = ograd.pearson_loss_grad(X.astype(np.float64), W)
    for precision in ("fp32", "bf16x3", "fp64"):
        g = _gpu_grad(X, W, gpu_device, precision)
        assert np.all(g[np.isnan(X)] == 0.0)
        err = np.abs(g - ref).max() / np.abs(ref).max()
        assert err <= 1e-4, (precision, err)


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
def test_backward_full_size(gpu_device, precision):
    case = synth.cfg_differentiation()
    X = case.X
    W = case.W
    print(f"[backward full size] {precision}", flush=True)
    _, ref, _ = ograd.pearson_loss_grad(X.astype(np.float64), W)
    g = _gpu_grad(X, W, gpu_device, precision)
    miss = np.isnan(X)
    assert np.all(g[miss] == 0.0)
    for (i, c) in case.nan_entries:
        assert g[i, c] == 0.0
    err = np.abs(g - ref).max() / np.abs(ref).max()
    assert err <= 1e-4, err
    # central finite differences of the FP64 loss, one column at a time
    Xd = X.astype(np.float64)
    h = 1e-3
    Wsym = W + W.T
    for (i, c) in case.fd_entries:
        xp = Xd.copy()
        xm = Xd.copy()
        xp[i, c] += h
        xm[i, c] -= h
        fd = (Wsym[c] * (_row_r(xp, c) - _row_r(xm, c))).sum() / (2 * h)
        assert abs(fd - g[i, c]) <= 1e-2 * max(abs(fd), 1e-3 * np.abs(ref).max()), (i, c, fd, g[i, c])
