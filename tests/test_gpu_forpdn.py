"""FORPDN on the device against the FP64 oracle (needs an MI355X).

Each case compares the noise estimate, the per-group thresholds (equal to the
oracle's, or a neighbouring grid point whose oracle SURE is within rounding of
the minimum) and the denoised cube element by element with the oracle run at
the device's thresholds.  Tolerances (relative Frobenius, element bound 10x):
FP64 1e-10, FP32 1e-5 -- the FP32 path rounds the wavelet sums and the
tridiagonal solve (condition up to 1 + 4 lam = 4e4 at the top of the grid;
an FP32 emulation of the solve stays below 4e-7 of the norm there).
"""
import sys

import numpy as np
import pytest

from oracle import forpdn_oracle as F
from paper_2204_06979_amd import synth

import parity_metrics as PM

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _api():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2204_06979_amd import api
    return api


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _grid_index(lam):
    return int(np.argmin(np.abs(np.log10(F.LAM_GRID) - np.log10(lam))))


def _group_coefficients(Y64, L, sigma):
    H, W, p = Y64.shape
    B = np.stack([F.HO.dwt2((Y64 / sigma)[:, :, b], L) for b in range(p)])
    return [B[:, a:b].T for a, b in F.group_slices(H, W, L)]


def _check_lambdas(Y64, L, sigma, lam_dev, lam_ref, sure_ref):
    """Device thresholds are the oracle's grid points (to the last bit of the
    power of ten), or others whose oracle SURE is within rounding of the minimum."""
    Cs = None
    for j in range(len(lam_ref)):
        np.testing.assert_allclose(lam_dev[j], F.LAM_GRID[_grid_index(lam_dev[j])], rtol=1e-15)
        if _grid_index(lam_dev[j]) == _grid_index(lam_ref[j]):
            continue
        Cs = Cs or _group_coefficients(Y64, L, sigma)
        s_dev = F.smoother_sure(Cs[j], lam_dev[j])
        say("   group", j, "device lam", lam_dev[j], "oracle", lam_ref[j], "SURE", s_dev, "min", sure_ref[j])
        assert s_dev - sure_ref[j] <= 1e-9 * max(1.0, abs(sure_ref[j])), (j, s_dev, sure_ref[j])


def _check_sure(sure_dev, sure_ref, Y64, L, sigma, rel):
    """SURE is a small difference of large sums for the coarse groups: its
    error is bounded relative to the group's energy ||C||^2."""
    energy = np.array([np.sum(C * C) for C in _group_coefficients(Y64, L, sigma)])
    err = np.abs(sure_dev - sure_ref)
    say("   SURE error / group energy", err / energy)
    assert np.all(err <= rel * energy), (sure_dev, sure_ref, energy)


CASES = {
    "c1-fp64": lambda: (synth.config_cube(1, keep_clean=False).Y, 3, 1e-10),
    "ragged-fp64": lambda: (synth.mixing_cube(33, 33, 27, 9, 3, 12.0, 2, dtype=np.float64,
                                              keep_clean=False).Y, 2, 1e-10),
    "ragged-fp32": lambda: (synth.mixing_cube(37, 37, 53, 17, 3, 12.0, 3, dtype=np.float32,
                                              keep_clean=False).Y, 3, 1e-5),
    "even-fp32": lambda: (synth.mixing_cube(97, 96, 128, 40, 4, (5, 20), 4, dtype=np.float32,
                                            keep_clean=False).Y, 4, 1e-5),
    "224-fp32": lambda: (synth.mixing_cube(224, 96, 80, 224, 6, 12.0, 3, dtype=np.float32,
                                           keep_clean=False).Y, 3, 1e-5),
}


@pytest.mark.parametrize("case", list(CASES))
def test_forpdn_matches_oracle(case):
    api = _api()
    Y, L, tol = CASES[case]()
    if case == "224-fp32":
        Y = Y + np.float32(1e-3) * np.random.default_rng(5).standard_normal(Y.shape).astype(np.float32)
    say("forpdn", case, Y.shape, Y.dtype, "L", L)
    X, info = api.forpdn(torch.tensor(Y, device="cuda"), L)
    assert int(info["status"].item()) & ~8 == 0
    Y64 = Y.astype(np.float64)
    ref = F.forpdn(Y64, L)
    sig = info["sigma"].cpu().numpy()
    np.testing.assert_allclose(sig, ref["sigma"], rtol=max(10 * tol, 1e-12))
    lam = info["lam"].cpu().numpy()
    say("   lam device", lam, "oracle", ref["lam"])
    _check_lambdas(Y64, L, ref["sigma"], lam, ref["lam"], ref["sure"])
    ref2 = F.forpdn(Y64, L, sigma=sig, lam=lam)
    _check_sure(info["sure"].cpu().numpy(), ref2["sure"], Y64, L, sig, 1e-12 if tol < 1e-9 else 1e-6)
    e, emax = PM.errors(X.cpu().numpy(), ref2["X"])
    say("   rel err", e, "max err / max", emax)
    PM.assert_close(X.cpu().numpy(), ref2["X"], tol, case)


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_forpdn_given_sigma_and_lambda(dtype):
    api = _api()
    cube = synth.config_cube(1, keep_clean=False)
    Y = cube.Y.astype(dtype)
    sig = cube.sigma_true
    lam = np.array([1e3, 10.0, 0.5, 1e-3])
    X, info = api.forpdn(torch.tensor(Y, device="cuda"), 3, sigma=torch.tensor(sig), lam=torch.tensor(lam))
    ref = F.forpdn(Y.astype(np.float64), 3, sigma=sig, lam=lam)
    tol = 1e-10 if dtype == np.float64 else 1e-5
    np.testing.assert_array_equal(info["sigma"].cpu().numpy(), sig)
    np.testing.assert_array_equal(info["lam"].cpu().numpy(), lam)
    _check_sure(info["sure"].cpu().numpy(), ref["sure"], Y.astype(np.float64), 3, sig,
                1e-12 if dtype == np.float64 else 1e-6)
    PM.assert_close(X.cpu().numpy(), ref["X"], tol, "given " + np.dtype(dtype).name)


def test_forpdn_strided_input_and_output():
    api = _api()
    cube = synth.mixing_cube(8, 40, 36, 20, 3, 12.0, 2, dtype=np.float32, keep_clean=False)
    H, W, p = cube.Y.shape
    big = torch.zeros(H, W + 2, 24, device="cuda")
    big[:, :W, :p] = torch.tensor(cube.Y, device="cuda")
    out = torch.full((H, W + 1, 22), 7.0, device="cuda")
    X, info = api.forpdn(big[:, :W, :p], 2, X=out[:, :W, :p])
    ref = F.forpdn(cube.Y.astype(np.float64), 2, sigma=info["sigma"].cpu().numpy(), lam=info["lam"].cpu().numpy())
    PM.assert_close(out[:, :W, :p].cpu().numpy(), ref["X"], 1e-5, "strided")
    assert bool((out[:, :W, p:] == 7.0).all()) and bool((out[:, W:] == 7.0).all())


def test_forpdn_full_size():
    """349 x 1905 x 144 FP32, 4 levels: the whole cube against the oracle at
    the device's noise estimate and thresholds, and each threshold no worse
    than its grid neighbours by the oracle's SURE."""
    api = _api()
    cube = synth.config_cube(2, keep_clean=False)
    Y = cube.Y
    H, W, p = Y.shape
    L = 4
    X, info = api.forpdn(torch.tensor(Y, device="cuda"), L)
    sig = info["sigma"].cpu().numpy()
    lam = info["lam"].cpu().numpy()
    say("   lam", lam)
    Y64 = Y.astype(np.float64)
    ref = F.forpdn(Y64, L, sigma=sig, lam=lam)
    _check_sure(info["sure"].cpu().numpy(), ref["sure"], Y64, L, sig, 1e-6)
    e, emax = PM.errors(X.cpu().numpy(), ref["X"])
    say("   rel err", e, "max err / max", emax)
    PM.assert_close(X.cpu().numpy(), ref["X"], 1e-5, "c2 forpdn")
    B = np.stack([F.HO.dwt2((Y64 / sig)[:, :, b], L) for b in range(p)])
    grid = list(F.LAM_GRID)
    for j, (a, b) in enumerate(F.group_slices(H, W, L)):
        k = _grid_index(lam[j])
        C = B[:, a:b].T
        here = F.smoother_sure(C, lam[j])
        for kk in (k - 1, k + 1):
            if 0 <= kk < len(grid):
                assert here <= F.smoother_sure(C, grid[kk]) + 1e-9 * abs(here), (j, kk)
