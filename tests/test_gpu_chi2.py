"""GPU parity of the chi-squared test (napy_chi2) against the FP64 oracle
(oracle/chi2.py) on seeded synthetic categorical matrices.

The contingency counts are exact integers on both sides and n must match
exactly; chi2 and V are FP64 sums of the same terms in a different order
(relative 1e-10); the oracle's p comes from SciPy's chi-squared tail, the
device's from its own incomplete gamma (pinned at 1e-12 against a 40-digit
reference in test_abi.py), so p agrees to 1e-9 relative.
"""

import numpy as np
import pytest

from oracle import chi2 as oc

pytestmark = pytest.mark.gpu


def _run(L, gpu_device, **kw):
    import torch
    import paper_2505_00448_amd as napy
    out = napy.chi2(torch.from_numpy(L).to(gpu_device), **kw)
    return tuple(out[k].cpu().numpy() for k in ("chi2", "p", "v", "n"))


def _check(got, ref, what):
    for name, g, r in zip(("chi2", "p", "v"), got[:3], ref[:3]):
        assert np.array_equal(np.isnan(g), np.isnan(r)), f"{what}: NaN placement of {name} differs"
        ok = ~np.isnan(r)
        tol = 1e-9 if name == "p" else 1e-10
        np.testing.assert_allclose(g[ok], r[ok], rtol=tol, atol=1e-12 if name != "p" else 1e-300,
                                   err_msg=f"{what} {name}")
    np.testing.assert_array_equal(got[3], ref[3], err_msg=f"{what} n")


def _with_edges(L, ncat):
    S = L.shape[0]
    one_cat = np.where(np.isnan(L[:, 0]), np.nan, 1.0)
    bad = L[:, 1].copy()
    bad[2] = ncat
    all_missing = np.full(S, np.nan)
    dup = L[:, 0].copy()  # perfect dependence on column 0
    return np.column_stack([L, one_cat, bad, all_missing, dup]).astype(np.float32)


@pytest.mark.parametrize("ncat,F", [(2, 30), (3, 50), (5, 41)])
def test_chi2_matches_oracle(gpu_device, ncat, F):
    import synth
    print(f"chi2 ncat={ncat} F={F}", flush=True)
    L = _with_edges(synth.categorical_matrix(900, F, ncat, seed=ncat * 100 + F), ncat)
    got = _run(L, gpu_device, ncat=ncat)
    ref = oc.chi2(L, ncat=ncat)
    _check(got, ref, f"ncat={ncat} F={F}")
    Fx = L.shape[1]
    np.testing.assert_array_equal(got[0], got[0].T)  # both triangles from one computation
    assert np.all(np.isnan(got[1][Fx - 4])) and np.all(got[3][Fx - 3] == 0)  # one category; invalid label


@pytest.mark.parametrize("shape", [(1, 1), (2, 3), (0, 4), (7, 22)])
def test_ragged_shapes(gpu_device, shape):
    import synth
    S, F = shape
    print(f"chi2 shape {shape}", flush=True)
    L = synth.categorical_matrix(max(S, 1), F, 3, missing=0.2, seed=S * 7 + F)[:S]
    _check(_run(L, gpu_device, ncat=3), oc.chi2(L, ncat=3), f"shape {shape}")


def test_sentinel_and_default_ncat(gpu_device):
    import synth
    print("chi2 sentinel", flush=True)
    L = synth.categorical_matrix(500, 9, 4, seed=77)
    Ls = np.where(np.isnan(L), -1.0, L).astype(np.float32)
    _check(_run(Ls, gpu_device, missing=-1.0), oc.chi2(L), "sentinel")


def test_full_size_sampled_pairs(gpu_device):
    """10,000 samples, 30% missing, 400 features with up to 4 categories; 300
    seeded pairs checked by the oracle."""
    import synth
    print("chi2 full size", flush=True)
    L = synth.categorical_matrix(10_000, 400, 4, seed=9)
    c2, p, v, n = _run(L, gpu_device, ncat=4)
    rng = np.random.default_rng(2)
    pairs = list(zip(rng.integers(0, 400, 300).tolist(), rng.integers(0, 400, 300).tolist()))
    ref = oc.chi2(L, ncat=4, pairs=pairs)
    gi = np.array([a for a, _ in pairs])
    hi = np.array([b for _, b in pairs])
    _check((c2[gi, hi], p[gi, hi], v[gi, hi], n[gi, hi]), ref, "full size")
    assert np.nanmin(p) < 1e-10  # dependent pairs exist (shared factors)
