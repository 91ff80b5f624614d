"""FP64 reference gradient of a weighted sum of the pairwise-deletion Pearson
matrix, by CPU autograd.

TEST INFRASTRUCTURE ONLY (imported by tests and the benchmark's CPU leg).

The paper has no gradient; this is the derivative of its Pearson definition
(Sections 3.2 and 3.5.2) with respect to the observed data.  For every pair
(g, h) the coefficient on I(g,h) is written with the pair means over I(g,h):

    r_gh = sum_I (x_g - a)(x_h - b) / sqrt(sum_I (x_g - a)^2 * sum_I (x_h - b)^2)

with a, b the means of x_g, x_h over I(g,h).  Expanding the sums over the
0/1 presence matrix M and the zero-filled data X0 turns every per-pair sum
into one matrix product, which lets autograd run over all pairs at once.  The
loss is L = sum_{g != h} W_gh r_gh over defined pairs only; the diagonal is
the constant 1 and undefined pairs (|I| <= 1 or zero variance) contribute
nothing (reading: the paper defines no value there, so no gradient flows).
Missing entries are not variables of the loss, so their gradient is zero.
"""

from __future__ import annotations

import numpy as np


def _pearson_torch(X0, M):
    import torch
    n = M.T @ M
    Sx = X0.T @ M            # [g, h]: sum over I(g,h) of x_g
    Sy = M.T @ X0            # [g, h]: sum over I(g,h) of x_h
    Sxx = (X0 * X0).T @ M
    Syy = M.T @ (X0 * X0)
    Sxy = X0.T @ X0
    nn = torch.clamp(n, min=1.0)
    a = Sx / nn
    b = Sy / nn
    cov = Sxy - a * Sy - b * Sx + nn * a * b
    vx = Sxx - 2 * a * Sx + nn * a * a
    vy = Syy - 2 * b * Sy + nn * b * b
    return n, cov, vx, vy


def pearson_loss_grad(X: np.ndarray, W: np.ndarray, var_rel_tol: float = 1e-12):
    """Returns (loss, dL/dX float64 [S, F] with zeros at missing entries,
    r float64 [F, F])."""
    import torch
    Xd = torch.from_numpy(np.asarray(X, dtype=np.float64).copy())
    present = ~torch.isnan(Xd)
    M = present.to(torch.float64)
    # centre each column by its observed mean first: r is shift invariant, so
    # this changes neither r nor its gradient, and keeps the sums well scaled
    mu = torch.nan_to_num(Xd).sum(0) / torch.clamp(M.sum(0), min=1.0)
    Xc = torch.where(present, Xd - mu, torch.zeros_like(Xd)).detach().requires_grad_(True)
    X0 = Xc * M
    n, cov, vx, vy = _pearson_torch(X0, M)
    F = Xd.shape[1]
    eye = torch.eye(F, dtype=torch.bool)
    Sxx = (X0 * X0).T @ M
    Syy = M.T @ (X0 * X0)
    valid = (n >= 2) & (vx > var_rel_tol * Sxx.detach()) & (vy > var_rel_tol * Syy.detach()) & ~eye
    den = torch.sqrt(torch.where(valid, vx * vy, torch.ones_like(vx)))
    r = torch.where(valid, cov / den, torch.zeros_like(cov))
    Wt = torch.from_numpy(np.asarray(W, dtype=np.float64))
    loss = (Wt * r).sum()
    loss.backward()
    g = Xc.grad.detach().numpy().copy()
    g[~present.numpy()] = 0.0
    return float(loss.detach()), g, r.detach().numpy()


def pearson_loss(X: np.ndarray, W: np.ndarray, var_rel_tol: float = 1e-12) -> float:
    """The loss alone in FP64 (for central finite differences)."""
    import torch
    with torch.no_grad():
        Xd = torch.from_numpy(np.asarray(X, dtype=np.float64).copy())
        present = ~torch.isnan(Xd)
        M = present.to(torch.float64)
        mu = torch.nan_to_num(Xd).sum(0) / torch.clamp(M.sum(0), min=1.0)
        X0 = torch.where(present, Xd - mu, torch.zeros_like(Xd))
        n, cov, vx, vy = _pearson_torch(X0, M)
        F = Xd.shape[1]
        eye = torch.eye(F, dtype=torch.bool)
        Sxx = (X0 * X0).T @ M
        Syy = M.T @ (X0 * X0)
        valid = (n >= 2) & (vx > var_rel_tol * Sxx) & (vy > var_rel_tol * Syy) & ~eye
        den = torch.sqrt(torch.where(valid, vx * vy, torch.ones_like(vx)))
        r = torch.where(valid, cov / den, torch.zeros_like(cov))
        return float((torch.from_numpy(np.asarray(W, dtype=np.float64)) * r).sum())
