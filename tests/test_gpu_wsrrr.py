"""WSRRR on the device against the FP64 oracle (needs an MI355X).

The oracle runs at the device's noise estimate and SURE thresholds (their
choice is tested with HyRes), so the comparison isolates the alternation:
the final subspace and the denoised cube, element by element.  Tolerances as
for HyRes (relative Frobenius; element bound 10x): FP64 1e-10, FP32 1e-5.
"""
import sys

import numpy as np
import pytest

from oracle import wsrrr_oracle as WS
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


CASES = {
    "c1-fp64": lambda: (synth.config_cube(1, keep_clean=False).Y, 4, 3, 5, 1e-10),
    "ragged-fp32": lambda: (synth.mixing_cube(97, 97, 133, 40, 4, 12.0, 3, dtype=np.float32,
                                              keep_clean=False).Y, 5, 3, 3, 1e-5),
    "dense-fp32": lambda: (synth.mixing_cube(98, 61, 75, 37, 4, 12.0, 3, dtype=np.float32,
                                             keep_clean=False).Y, 4, 3, 3, 1e-5),
    "c2-fp32": lambda: (synth.config_cube(2, keep_clean=False).Y, 8, 4, 3, 1e-5),
}


@pytest.mark.parametrize("case", list(CASES))
def test_wsrrr_matches_oracle(case):
    api = _api()
    Y, r, L, K, tol = CASES[case]()
    say("wsrrr", case, Y.shape, Y.dtype, "r", r, "L", L, "iterations", K)
    X, info = api.wsrrr(torch.tensor(Y, device="cuda"), r, L, K)
    assert int(info["status"].item()) & ~8 == 0
    sig = info["sigma"].cpu().numpy()
    lam = info["lam"].cpu().numpy()
    ref = WS.wsrrr(Y.astype(np.float64), r, L, K, sigma=sig, lam=lam)
    V = info["V"].cpu().numpy()
    cosines = np.linalg.svd(V.T @ ref["V"], compute_uv=False)
    say("   subspace min cosine", cosines.min(), "V max abs diff", np.abs(V - ref["V"]).max())
    assert np.abs(V - ref["V"]).max() <= (1e-9 if tol < 1e-9 else 1e-3)
    e, emax = PM.errors(X.cpu().numpy(), ref["X"])
    say("   rel err", e, "max err / max", emax)
    PM.assert_close(X.cpu().numpy(), ref["X"], tol, case)


def test_wsrrr_without_iterations_is_the_hyres_solve():
    api = _api()
    cube = synth.mixing_cube(5, 64, 80, 24, 3, 12.0, 3, dtype=np.float32, keep_clean=False)
    Yt = torch.tensor(cube.Y, device="cuda")
    X0, _ = api.wsrrr(Yt, 4, 3, 0)
    X1, _ = api.denoise(Yt, 4, 3)
    assert torch.equal(X0, X1)


def test_wsrrr_strided_input():
    """A window of a larger tensor (strided pixels) gives the contiguous result."""
    api = _api()
    cube = synth.mixing_cube(99, 45, 70, 28, 3, 12.0, 3, dtype=np.float32, keep_clean=False)
    H, W, p = cube.Y.shape
    big = torch.zeros(H, W + 2, p + 3, device="cuda")
    big[:, :W, :p] = torch.tensor(cube.Y, device="cuda")
    Xs, info = api.wsrrr(big[:, :W, :p], 4, 3, 3)
    ref = WS.wsrrr(cube.Y.astype(np.float64), 4, 3, 3, sigma=info["sigma"].cpu().numpy(),
                   lam=info["lam"].cpu().numpy())
    PM.assert_close(Xs.cpu().numpy(), ref["X"], 1e-5, "strided")
