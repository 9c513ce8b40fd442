"""hyres_denoise_noalloc (scratch from the library's per-device array) against
hyres_denoise (caller workspace) on the same cubes: two calls in a row, the
second on a smaller cube, so the second runs over the first call's leftovers.

X, sigma, V, eigenvalues and thresholds must be bitwise equal (same kernels,
same launch sequence, same reduction orders); the SURE minima to rounding;
each result is also held to the oracle's tolerance."""
import ctypes as C
import sys

import numpy as np
import pytest
import torch

from paper_2204_06979_amd import _lib as L
from paper_2204_06979_amd import api, synth
from oracle import hyres_oracle as O
import parity_metrics as PM

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a)
    sys.stdout.flush()


def _cube(H, W, p, r, L_, seed):
    cube = synth.mixing_cube(seed, H, W, p, min(r, 6), 12.0, L_, dtype=np.float32, keep_clean=False)
    return cube.Y


@pytest.mark.parametrize("precision", ["native", "mixed"])
def test_noalloc_matches_workspace_entry_point(precision):
    cases = [(160, 224, 103, 7, 4, 11), (64, 96, 40, 5, 3, 12)]      # second call smaller
    for (H, W, p, r, Lv, seed) in cases:
        say("noalloc", precision, (H, W, p), "r", r, "L", Lv)
        Y = _cube(H, W, p, r, Lv, seed)
        Yt = torch.tensor(Y, device="cuda")
        Xa, ia = api.denoise(Yt, r, Lv, precision=precision)
        Xb, ib = api.denoise_noalloc(Yt, r, Lv, precision=precision)
        torch.cuda.synchronize()
        assert int(ib["status"].cpu()[0]) & ~8 == 0
        assert torch.equal(Xa, Xb), float((Xa - Xb).abs().max())
        for k in ("sigma", "V", "lam", "gap"):
            assert torch.equal(ia[k], ib[k]), k
        # the SURE minima are FP64 sums that the histogram pass forms with device
        # atomics: their last bits depend on the order the blocks arrive in
        torch.testing.assert_close(ia["sure"], ib["sure"], rtol=1e-12, atol=0.0)
        assert torch.equal(ia["evals"][: r + 1], ib["evals"][: r + 1])
        ref = O.hyres(Y.astype(np.float64), r, Lv, lam=ib["lam"].cpu().numpy())
        tol = PM.TOL["mixed" if precision == "mixed" else "float32"]
        fro, mx = PM.assert_close(Xb.cpu().numpy(), ref["X"], tol, "noalloc")
        say("   bitwise equal to hyres_denoise; vs oracle", fro, mx)


def test_noalloc_rejects_a_solve_beyond_its_scratch():
    lib = L.lib()
    opt = L.Options(12, 4, L.PREC_NATIVE, L.SCOPE_ALL, 0)
    nb = C.c_size_t()
    H, W, p = 1024, 1024, 128
    L.check(lib.hyres_denoise_workspace_size(H, W, p, C.byref(opt), L.HYRES_F32, C.byref(nb)))
    assert nb.value > L.NOALLOC_SCRATCH_BYTES
    Y = torch.zeros(H, W, p, dtype=torch.float32, device="cuda")
    X = torch.empty_like(Y)
    out = L.Outputs()
    st = lib.hyres_denoise_noalloc(api._handle(Y.device), Y.data_ptr(), H, W, p, p, W * p, L.HYRES_F32,
                                   C.byref(opt), None, None, X.data_ptr(), p, W * p, C.byref(out),
                                   api._stream(Y.device))
    assert st == 4      # HYRES_E_WORKSPACE, nothing enqueued
