"""HyMiNoR on the device against the FP64 oracle (needs an MI355X).

The sparse-noise stage is compared element by element with the oracle's
split-Bregman iteration on the same input, for band counts that take every
lane layout of the kernel (one, two or four lanes per pixel, ragged last
segments, pixel counts that leave a partial block), in FP64 and FP32; then
HyMiNoR end to end on the 64 x 64 x 32 FP64 cube and an FP32 cube with dead
columns, and at the 349 x 1905 x 144 FP32 size on sampled pixels.

Tolerances (relative Frobenius, element bound 10x as for HyRes): FP64 1e-10;
FP32 1e-5.  Each sweep is a contraction-free but non-expansive map of the
rounding error, so FP32 errors grow at most linearly with the sweep count: at
50 sweeps the FP32 emulation of the same recurrences stays near 2e-7 of the
norm and 2e-6 of the largest value.
"""
import sys

import numpy as np
import pytest

from oracle import hyminor_oracle as HM
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


def _spectra(seed, H, W, p, dtype):
    """Smooth spectra (random walks) with one-band spikes and dips on 3% of the voxels."""
    rng = np.random.default_rng(seed)
    h = 1.0 + 0.1 * np.cumsum(rng.standard_normal((H, W, p)), axis=2)
    mask = rng.random((H, W, p)) < 0.03
    h[mask] += rng.choice([-1.5, 2.0], size=int(mask.sum()))
    return h.astype(dtype)


F32_P = [1, 2, 17, 64, 65, 100, 128, 129, 144, 161, 191, 224]
F64_P = [1, 5, 32, 33, 96, 97, 150, 224]


@pytest.mark.parametrize("dtype,p", [(np.float32, p) for p in F32_P] + [(np.float64, p) for p in F64_P])
def test_l1l1_matches_oracle(dtype, p):
    api = _api()
    H, W = 13, 29                    # 377 pixels: a partial block for every lane layout
    say("l1l1", dtype.__name__, "p", p)
    h = _spectra(p, H, W, p, dtype)
    lam, mu1, mu2, K = 0.7, 1.0, 0.5, 30
    X = api.l1l1_spectral(torch.tensor(h, device="cuda"), lam, mu1, mu2, K).cpu().numpy()
    ref = HM.l1l1_split_bregman(h.astype(np.float64), lam, mu1, mu2, K)
    tol = 1e-10 if dtype == np.float64 else 1e-5
    e, emax = PM.errors(X, ref)
    say("   rel err", e, "max err / max", emax, "changed voxels", int((np.abs(ref - h) > 1e-3).sum()))
    PM.assert_close(X, ref, tol, "l1l1 p=%d" % p)


def test_l1l1_in_place_and_strided():
    api = _api()
    H, W, p = 21, 40, 37
    h = _spectra(5, H, W, p, np.float32)
    ref = HM.l1l1_split_bregman(h.astype(np.float64), 0.8, 2.0, 1.0, 20)
    # padded pixels (pitch 40) and padded rows, result in a buffer of another layout
    big = torch.zeros(H, W + 3, 40, device="cuda")
    big[:, :W, :p] = torch.tensor(h, device="cuda")
    src = big[:, :W, :p]
    X1 = api.l1l1_spectral(src, 0.8, 2.0, 1.0, 20)
    PM.assert_close(X1.cpu().numpy(), ref, 1e-5, "strided")
    # in place on the padded buffer: the padding is left alone
    X2 = api.l1l1_spectral(src, 0.8, 2.0, 1.0, 20, X=src)
    assert X2.data_ptr() == src.data_ptr()
    np.testing.assert_array_equal(src.cpu().numpy(), X1.cpu().numpy())
    assert not big[:, :W, p:].any() and not big[:, W:].any()


def test_l1l1_rejects_bad_options():
    api = _api()
    from paper_2204_06979_amd import _lib as L
    h = torch.zeros(4, 4, 8, device="cuda")
    for lam, mu1, mu2, k in [(1.0, 0.0, 1.0, 5), (1.0, 1.0, -1.0, 5), (-0.1, 1.0, 1.0, 5), (1.0, 1.0, 1.0, 0),
                             (float("nan"), 1.0, 1.0, 5)]:
        with pytest.raises(RuntimeError, match="HYRES_E_SHAPE"):
            api.l1l1_spectral(h, lam, mu1, mu2, k)
    # in place with another layout
    with pytest.raises(RuntimeError, match="HYRES_E_SHAPE"):
        o = L.L1Options(1.0, 1.0, 1.0, 3)
        st = L.lib().hyres_l1l1_spectral(api._handle(h.device), h.data_ptr(), 4, 4, 8, 8, 32, L.HYRES_F32,
                                         L.C.byref(o), h.data_ptr(), 8, 40, api._stream(h.device))
        L.check(st, "in place, other layout")


@pytest.mark.parametrize("case", ["c1-fp64", "dead-columns-fp32"])
def test_hyminor_matches_oracle(case):
    """End to end against the oracle at the device's HyRes thresholds, and
    stage by stage: hyres_hyminor equals HyRes followed by the stage bit for
    bit; HyRes meets its own bar; the stage on the device's HyRes output
    meets the stage's bar element by element.  (The FP32 end-to-end element
    error is larger than either stage's: at rank 8 on a rank-3 cube HyRes
    carries ill-determined noise components whose FP32 rounding the l1-l1
    stage moves between nearby piecewise-linear pieces; the norm stays at
    the FP32 bar.)"""
    api = _api()
    if case == "c1-fp64":
        cube = synth.config_cube(1, keep_clean=False)
        Y, r, L, tol = cube.Y, 4, 3, 1e-10
    else:
        cube = synth.mixing_cube(31, 96, 80, 40, 3, 20.0, 3, dtype=np.float32, keep_clean=False,
                                 dead_columns=True)
        Y, r, L, tol = cube.Y, 8, 3, 1e-5
    lam, mu1, mu2, K = 0.55, 1.0, 1.0, 50
    say("hyminor", case, Y.shape, Y.dtype)
    Yt = torch.tensor(Y, device="cuda")
    X, info = api.hyminor(Yt, r, L, lam, mu1, mu2, K)
    assert int(info["status"].item()) & ~8 == 0
    X1, _ = api.denoise(Yt, r, L)
    X2 = api.l1l1_spectral(X1, lam, mu1, mu2, K)
    assert torch.equal(X, X2)
    # the oracle at the device's thresholds (their SURE choice is tested with HyRes)
    ref = HM.hyminor(Y.astype(np.float64), r, L, lam, mu1, mu2, K, hyres_lam=info["lam"].cpu().numpy())
    e, emax = PM.errors(X.cpu().numpy(), ref["X"])
    say("   end to end rel err", e, "max err / max", emax)
    assert e <= tol
    PM.assert_close(X1.cpu().numpy(), ref["X_hyres"], tol, case + " HyRes stage")
    h = X1.cpu().numpy().astype(np.float64)
    ref2 = HM.l1l1_split_bregman(h, lam, mu1, mu2, K)
    e2, emax2 = PM.errors(X.cpu().numpy(), ref2)
    say("   sparse stage on the device's HyRes output: rel err", e2, "max err / max", emax2)
    PM.assert_close(X.cpu().numpy(), ref2, tol, case + " sparse stage")
    if case == "c1-fp64":
        PM.assert_close(X.cpu().numpy(), ref["X"], tol, case)


def test_hyminor_full_size_sampled():
    """349 x 1905 x 144 FP32, rank 8: hyres_hyminor equals HyRes followed by
    the stage bit for bit, and the stage matches the oracle on 3000 sampled
    pixels of the device's HyRes output (the stage is per pixel)."""
    api = _api()
    cube = synth.config_cube(2, keep_clean=False)
    Yt = torch.tensor(cube.Y, device="cuda")
    lam, mu1, mu2, K = 0.55, 1.0, 1.0, 50
    X, _ = api.hyminor(Yt, 8, 4, lam, mu1, mu2, K)
    X1, _ = api.denoise(Yt, 8, 4)
    X2 = api.l1l1_spectral(X1, lam, mu1, mu2, K)
    assert torch.equal(X, X2)
    H, W, p = cube.Y.shape
    rng = np.random.default_rng(2)
    idx = rng.choice(H * W, 3000, replace=False)
    h = X1.reshape(H * W, p)[torch.tensor(idx, device="cuda")].cpu().numpy().astype(np.float64)
    got = X2.reshape(H * W, p)[torch.tensor(idx, device="cuda")].cpu().numpy()
    ref = HM.l1l1_split_bregman(h, lam, mu1, mu2, K)
    e, emax = PM.errors(got, ref)
    say("   sampled rel err", e, "max err / max", emax)
    PM.assert_close(got, ref, 1e-5, "hyminor c2 sampled")
