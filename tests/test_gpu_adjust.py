"""GPU parity of the multiple-testing correction (napy_adjust_pvalues) against
the FP64 oracle (oracle/adjust.py) on seeded synthetic p matrices.

The device path forms the same FP64 products and quotients as the oracle
(factor * p / k, then minima), so Bonferroni and Benjamini-Hochberg agree bit
for bit; Benjamini-Yekutieli's factor m c(m) is summed differently (exactly
rounded in the oracle, a direct sum or the asymptotic expansion on the
device), so it agrees to a relative 1e-13.
"""

import numpy as np
import pytest

from oracle import adjust as oadj

pytestmark = pytest.mark.gpu


def p_matrix(F, seed, nan_frac=0.02, tie_frac=0.2):
    import synth
    return synth.pvalue_matrix(F, seed=seed, nan_frac=nan_frac, tie_frac=tie_frac)


def _check(got, ref, method, what):
    assert np.array_equal(np.isnan(got), np.isnan(ref)), f"{what}: NaN placement differs"
    ok = ~np.isnan(ref)
    if method == "by":
        np.testing.assert_allclose(got[ok], ref[ok], rtol=1e-13, atol=0, err_msg=what)
    else:
        np.testing.assert_array_equal(got[ok], ref[ok], err_msg=what)


@pytest.mark.parametrize("method", ["bonferroni", "bh", "by"])
@pytest.mark.parametrize("F", [1, 2, 3, 50, 91, 92, 257, 1000, 2049])
def test_adjust_matches_oracle(gpu_device, F, method):
    import torch
    import paper_2505_00448_amd as napy
    print(f"adjust F={F} method={method}", flush=True)
    P = p_matrix(F, 100 + F)
    got = napy.adjust_pvalues(torch.from_numpy(P).to(gpu_device), method).cpu().numpy()
    ref = oadj.adjust_matrix(P, method)
    _check(got, ref, method, f"F={F} {method}")


@pytest.mark.parametrize("method", ["bh", "by"])
def test_adjust_full_size_4000(gpu_device, method):
    """Largest configuration of the benchmarks: 4,000 variables (8.0 M pairs)."""
    import torch
    import paper_2505_00448_amd as napy
    print(f"adjust F=4000 method={method}", flush=True)
    P = p_matrix(4000, 4000, nan_frac=0.001, tie_frac=0.05)
    got = napy.adjust_pvalues(torch.from_numpy(P).to(gpu_device), method).cpu().numpy()
    _check(got, oadj.adjust_matrix(P, method), method, f"F=4000 {method}")


def test_adjust_in_place_strided_and_edge_cases(gpu_device):
    import torch
    import paper_2505_00448_amd as napy
    print("adjust in place / strided / all-NaN / all-equal", flush=True)
    F = 300
    P = p_matrix(F, 7)
    ref = oadj.adjust_matrix(P, "bh")
    # in place
    T = torch.from_numpy(P.copy()).to(gpu_device)
    napy.adjust_pvalues(T, "bh", out=T)
    _check(T.cpu().numpy(), ref, "bh", "in place")
    # leading dimension larger than F on both sides
    big = torch.full((F, F + 37), 7.0, dtype=torch.float64, device=gpu_device)
    big[:, :F] = torch.from_numpy(P).to(gpu_device)
    outb = torch.full((F, F + 5), -3.0, dtype=torch.float64, device=gpu_device)
    napy.adjust_pvalues(big[:, :F], "bh", out=outb[:, :F])
    _check(outb[:, :F].cpu().numpy(), ref, "bh", "strided")
    assert bool((outb[:, F:] == -3.0).all()), "wrote past the F columns"
    # every pair undefined: m = 0
    A = np.full((5, 5), np.nan)
    got = napy.adjust_pvalues(torch.from_numpy(A).to(gpu_device), "by").cpu().numpy()
    assert np.all(np.isnan(got))
    # all pairs equal: BH leaves them, Bonferroni multiplies by m
    E = np.full((40, 40), 1e-5)
    for method in ("bh", "bonferroni", "by"):
        got = napy.adjust_pvalues(torch.from_numpy(E).to(gpu_device), method).cpu().numpy()
        _check(got, oadj.adjust_matrix(E, method), method, f"all-equal {method}")


def test_adjust_repeat_calls_deterministic(gpu_device):
    import torch
    import paper_2505_00448_amd as napy
    print("adjust determinism", flush=True)
    P = torch.from_numpy(p_matrix(700, 9)).to(gpu_device)
    ws = torch.empty(napy._lib.load().napy_adjust_workspace(700), dtype=torch.uint8, device=gpu_device)
    a = napy.adjust_pvalues(P, "by", workspace=ws)
    b = napy.adjust_pvalues(P, "by", workspace=ws)
    assert torch.equal(torch.nan_to_num(a, nan=-1.0), torch.nan_to_num(b, nan=-1.0))
