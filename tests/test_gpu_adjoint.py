"""Hand-written adjoint of the solve and the SURE derivative (needs an MI355X).

The adjoint is checked three ways: against central finite differences of the
device's own FP64 forward (32 x 32 x 16 sub-cube, step 1e-6), against torch
autograd through the FP64 CPU oracle forward, and, at the 256 x 256 x 191
FP32 workload, against that oracle gradient at the FP32 tolerance.
"""
import sys

import numpy as np
import pytest

from oracle import hyres_oracle as O
from paper_2204_06979_amd import synth

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


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _oracle_grad(Y, lam, r, L, V_ref, R):
    from oracle import grad as OG
    Yt = torch.tensor(Y, dtype=torch.float64, requires_grad=True)
    lt = torch.tensor(lam, dtype=torch.float64, requires_grad=True)
    X = OG.hyres_forward(Yt, lt, r, L, sign_ref=torch.tensor(V_ref, dtype=torch.float64))
    (X * torch.tensor(R, dtype=torch.float64)).sum().backward()
    return Yt.grad.numpy(), lt.grad.numpy()


def test_sure_grad_matches_definition():
    api = _api()
    rng = np.random.default_rng(4)
    b = np.stack([rng.standard_normal(40000), rng.normal(0, 3, 40000), rng.laplace(0, 1, 40000)])
    lam = np.array([0.731, 2.05, 1.3])
    for dt in (np.float64, np.float32):
        bb = b.astype(dt)
        g = api.sure_grad(torch.tensor(bb, device="cuda"), torch.tensor(lam)).cpu().numpy()
        for i in range(3):
            x = np.abs(bb[i].astype(np.float64))
            cnt = int(np.sum(x > np.float64(dt(lam[i]))))
            assert g[i] == 2.0 * lam[i] * cnt
            h = 1e-7
            fd = (O.sure_at(bb[i].astype(np.float64), lam[i] + h) - O.sure_at(bb[i].astype(np.float64), lam[i] - h)) / (2 * h)
            assert abs(fd - g[i]) <= 1e-5 * abs(g[i]), (fd, g[i])


def _setup(dtype, H, W, p, r, L, seed=4):
    c = synth.mixing_cube(seed, H, W, p, r, 10.0, L, dtype=np.float64, keep_clean=False)
    Y = (c.Y + 1e-3 * np.random.default_rng(seed).standard_normal(c.Y.shape)).astype(dtype)
    ref = O.hyres(Y.astype(np.float64), r, L)
    lam = ref["lam"] * 0.8 + 0.02
    return Y, lam, ref


def test_adjoint_against_finite_differences_fp64():
    api = _api()
    cube = synth.config_cube(4, keep_clean=False)
    Y = cube.Y[:32, :32, :16].astype(np.float64)
    r, L = 6, 3
    ref = O.hyres(Y, r, L)
    lam = ref["lam"] * 0.8 + 0.02
    rng = np.random.default_rng(7)
    R = rng.standard_normal(Y.shape)
    Yt = torch.tensor(Y, device="cuda", requires_grad=True)
    lt = torch.tensor(lam, device="cuda", requires_grad=True)
    X = api.HyResFunction.apply(Yt, lt, r, L, "native")
    loss = (X * torch.tensor(R, device="cuda")).sum()
    loss.backward()
    gY = Yt.grad.cpu().numpy()
    gl = lt.grad.cpu().numpy()

    def f(Yv, lv):
        Xv, _ = api.denoise(torch.tensor(Yv, device="cuda"), r, L, lam=torch.tensor(lv))
        Xv = Xv.cpu().numpy()
        return float((Xv * R).sum()), float(np.abs(Xv * R).sum())

    # a central difference carries the truncation error O(h^2) and the
    # rounding of the two evaluations, about 1e-15 sum|R X| / h; the
    # comparison allows that plus 1e-5 relative
    h = 1e-6
    for k in range(6):
        E = rng.standard_normal(Y.shape)
        E /= np.linalg.norm(E)
        (fp, mag), (fm, _) = f(Y + h * E, lam), f(Y - h * E, lam)
        fd = (fp - fm) / (2 * h)
        an = float((gY * E).sum())
        say("  dir", k, "fd", fd, "adjoint", an)
        assert abs(fd - an) <= 1e-5 * abs(an) + 1e-15 * mag / h
    for i in range(r):
        e = np.zeros(r)
        e[i] = h
        (fp, mag), (fm, _) = f(Y, lam + e), f(Y, lam - e)
        fd = (fp - fm) / (2 * h)
        say("  lambda", i, "fd", fd, "adjoint", gl[i])
        assert abs(fd - gl[i]) <= 1e-5 * abs(gl[i]) + 1e-15 * mag / h


@pytest.mark.parametrize("H,W,p,r,L", [(64, 64, 32, 4, 3), (37, 53, 20, 3, 2)])
def test_adjoint_matches_oracle_autograd_fp64(H, W, p, r, L):
    api = _api()
    Y, lam, ref = _setup(np.float64, H, W, p, r, L)
    R = np.random.default_rng(1).standard_normal(Y.shape)
    dn = api.Denoiser(H, W, p, r, L, dtype=torch.float64)
    Yt = torch.tensor(Y, device="cuda")
    dn.run(Yt, None, torch.tensor(lam, device="cuda"))
    dY, dlam, st = api.denoise_backward(dn, Yt, torch.tensor(R, device="cuda"))
    assert int(st.cpu()[0]) == 0
    gY, gl = _oracle_grad(Y, lam, r, L, dn.V.T.cpu().numpy(), R)
    e = rel(dY.cpu().numpy(), gY)
    el = rel(dlam.cpu().numpy(), gl)
    say("  dY rel err", e, "dlambda rel err", el)
    assert e <= 1e-9 and el <= 1e-9


def test_adjoint_config4_fp32_against_oracle_gradient():
    api = _api()
    cube = synth.config_cube(4, keep_clean=False)
    Y = cube.Y
    H, W, p = Y.shape
    r, L = 6, 4
    Yt = torch.tensor(Y, device="cuda", requires_grad=True)
    # The soft threshold has a kink where |b| = lambda, and a SURE threshold is
    # one of the coefficients, sitting exactly on it.  The gradient is checked
    # at thresholds away from every kink: near each oracle SURE threshold, the
    # middle of the widest gap between the 32 nearest coefficient magnitudes.
    _, info = api.denoise(Yt.detach(), r, L)
    ref = O.hyres(Y.astype(np.float64), r, L)
    lam_np = np.empty(r)
    for k in range(r):
        a = np.sort(np.abs(ref["B"][k]))
        i0 = int(np.searchsorted(a, ref["lam"][k]))
        w = a[max(0, i0 - 16):i0 + 16]
        g = int(np.argmax(np.diff(w)))
        lam_np[k] = 0.5 * (w[g] + w[g + 1])
    lam = torch.tensor(lam_np, device="cuda")
    lt = lam.clone().requires_grad_(True)
    R = np.random.default_rng(2).standard_normal(Y.shape).astype(np.float32)
    X = api.HyResFunction.apply(Yt, lt, r, L, "native")
    (X * torch.tensor(R, device="cuda")).sum().backward()
    V = info["V"].cpu().numpy()
    say("config4 oracle gradient", Y.shape)
    Y64 = Y.astype(np.float64)
    gY, gl = _oracle_grad(Y64, lam.cpu().numpy(), r, L, V, R.astype(np.float64))
    # the tolerance is the oracle gradient's own sensitivity to FP32-level
    # perturbations of its input (relative 6e-8 per voxel): thresholded
    # coefficients that sit that close to lambda switch between kept and
    # zeroed, which moves the gradient far more than the FP32 rounding of
    # the adjoint's own arithmetic
    Yp = Y64 * (1.0 + 6e-8 * np.random.default_rng(9).standard_normal(Y.shape))
    gYp, glp = _oracle_grad(Yp, lam.cpu().numpy(), r, L, V, R.astype(np.float64))
    s_y, s_l = rel(gYp, gY), rel(glp, gl)
    e = rel(Yt.grad.cpu().numpy(), gY)
    el = rel(lt.grad.cpu().numpy(), gl)
    say("  dY rel err", e, "dlambda rel err", el, "oracle spread", s_y, s_l)
    assert e <= max(1e-4, 2.0 * s_y) and el <= max(1e-4, 2.0 * s_l)


def _midgap_lambda(B, lam):
    """A threshold near each SURE threshold but away from every kink: the
    middle of the widest gap between the 32 coefficient magnitudes nearest it."""
    out = np.empty(len(lam))
    for k in range(len(lam)):
        a = np.sort(np.abs(B[k]))
        i0 = int(np.searchsorted(a, lam[k]))
        w = a[max(0, i0 - 16):i0 + 16]
        g = int(np.argmax(np.diff(w)))
        out[k] = 0.5 * (w[g] + w[g + 1])
    return out


# FP32 cubes on each load path of the pixel products: 16-byte vectors (p % 4
# == 0), dense rows (odd p), strided pixels (a window of a larger tensor);
# pixel counts that do not fill the last 64-pixel tile
@pytest.mark.parametrize("H,W,p,r,L,layout", [(64, 64, 32, 4, 3, "vec"), (37, 53, 20, 3, 2, "vec"),
                                              (37, 53, 21, 3, 2, "dense"), (40, 45, 24, 4, 2, "strided"),
                                              (33, 70, 150, 5, 2, "dense")])
def test_adjoint_fp32_layouts_against_oracle_gradient(H, W, p, r, L, layout):
    api = _api()
    c = synth.mixing_cube(11, H, W, p, r, 10.0, L, dtype=np.float32, keep_clean=False)
    Y = c.Y
    Y64 = Y.astype(np.float64)
    ref = O.hyres(Y64, r, L)
    lam = _midgap_lambda(ref["B"], ref["lam"])
    say("fp32 adjoint", layout, Y.shape, "r", r, "L", L)
    if layout == "strided":
        big = torch.zeros(H, W + 3, p + 5, device="cuda")
        big[:, :W, :p] = torch.tensor(Y, device="cuda")
        Yt = big[:, :W, :p]
    else:
        Yt = torch.tensor(Y, device="cuda")
    R = np.random.default_rng(3).standard_normal(Y.shape).astype(np.float32)
    dn = api.Denoiser(H, W, p, r, L, dtype=torch.float32)
    dn.run(Yt, None, torch.tensor(lam, device="cuda"))
    dY, dlam, st = api.denoise_backward(dn, Yt, torch.tensor(R, device="cuda"))
    assert int(st.cpu()[0]) == 0
    gY, gl = _oracle_grad(Y64, lam, r, L, dn.V.T.cpu().numpy(), R.astype(np.float64))
    e = rel(dY.cpu().numpy(), gY)
    el = rel(dlam.cpu().numpy(), gl)
    say("  dY rel err", e, "dlambda rel err", el)
    assert e <= 1e-4 and el <= 1e-4
