"""Parity of the HIP path with the FP64 CPU oracle (needs an MI355X).

Tolerances: FP64 cubes <= 1e-10 relative (Frobenius), FP32 cubes <= 1e-5
relative; wavelet coefficients FP64 <= 1e-13 and FP32 <= 1e-6 relative to the
largest magnitude.  Where the device's rounding makes another near-optimal
candidate the SURE minimiser, it is accepted by the rule in sure_protocol.py
and the cube is then compared with the oracle run at the device's thresholds.
"""
import math
import sys

import numpy as np
import pytest

from oracle import hyres_oracle as O
from paper_2204_06979_amd import synth

import parity_metrics as PM
import sure_protocol as SP

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


# ------------------------------------------------------------------ wavelets
@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("H,W,L,B", [(64, 64, 3, 2), (37, 53, 3, 3), (349, 191, 4, 2), (4, 9, 1, 1),
                                     (130, 517, 4, 1)])
def test_dwt2_matches_oracle(dtype, H, W, L, B):
    api = _api()
    say("dwt2", H, W, L, B, dtype.__name__)
    rng = np.random.default_rng(H * 1000 + W)
    x = rng.standard_normal((B, H, W)).astype(dtype)
    xt = torch.tensor(x, device="cuda")
    c = api.dwt2(xt, L)
    ref = np.stack([O.dwt2(x[b].astype(np.float64), L) for b in range(B)])
    got = c.cpu().numpy().astype(np.float64)
    tol = 1e-13 if dtype == np.float64 else 1e-6
    assert np.abs(got - ref).max() <= tol * np.abs(ref).max()
    # perfect reconstruction on the device
    xr = api.idwt2(c, H, W, L)
    tolr = 1e-13 if dtype == np.float64 else 2e-6
    assert np.abs(xr.cpu().numpy() - x).max() <= tolr * np.abs(x).max()


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_idwt2_with_threshold_matches_oracle(dtype):
    api = _api()
    rng = np.random.default_rng(7)
    H, W, L, B = 75, 98, 3, 3
    c = rng.standard_normal((B, O.coeff_count(H, W, L))).astype(dtype)
    lam = np.array([0.0, 0.7, 1.9])
    for scope in ("all", "detail"):
        got = api.idwt2(torch.tensor(c, device="cuda"), H, W, L, torch.tensor(lam), scope=scope).cpu().numpy()
        hL, wL = O.level_shapes(H, W, L)[-1]
        for b in range(B):
            cb = O.soft_threshold(c[b].astype(np.float64), lam[b])
            if scope == "detail":
                cb[-hL * wL:] = c[b, -hL * wL:]
            ref = O.idwt2(cb, H, W, L)
            tol = 1e-13 if dtype == np.float64 else 2e-6
            assert np.abs(got[b] - ref).max() <= tol * max(1.0, np.abs(ref).max())


# ---------------------------------------------------------------------- SURE
def _sure_cases():
    rng = np.random.default_rng(11)
    cases = []
    cases.append(("noise+signal", np.concatenate([rng.standard_normal(60000),
                                                  rng.normal(0, 6, 3000)])))
    cases.append(("tiny", rng.standard_normal(7)))
    cases.append(("one", np.array([2.5])))
    cases.append(("zeros", np.zeros(1000)))
    cases.append(("ties", np.round(rng.standard_normal(20000), 1)))
    cases.append(("all-large", rng.normal(0, 50, 5000)))
    cases.append(("ragged", rng.standard_normal(16384 * 3 + 17) * 0.3))
    return cases


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_sure_threshold_matches_oracle(dtype):
    api = _api()
    for name, b in _sure_cases():
        say("sure", name, dtype.__name__)
        bb = b.astype(dtype)
        lam, smin, st = api.sure_threshold(torch.tensor(bb[None, :], device="cuda"))
        lam = float(lam.cpu()[0])
        smin = float(smin.cpu()[0])
        lo, so = O.sure_threshold(bb.astype(np.float64))
        assert int(st.cpu()[0]) == 0, name
        assert lam == lo, (name, lam, lo)
        assert abs(smin - so) <= 1e-9 * max(1.0, abs(so)), (name, smin, so)


def test_sure_batched_rows_with_stride():
    api = _api()
    rng = np.random.default_rng(3)
    B, N = 5, 30001
    x = rng.standard_normal((B, N + 100)).astype(np.float32) * np.array([0.5, 1, 2, 4, 8])[:, None]
    t = torch.tensor(x, device="cuda")[:, :N]
    lam, smin, st = api.sure_threshold(t)
    for i in range(B):
        lo, so = O.sure_threshold(x[i, :N].astype(np.float64))
        assert float(lam[i]) == lo


# ------------------------------------------------------- noise and subspace
@pytest.mark.parametrize("cfg,tol", [(1, 1e-12), (4, 1e-5)])
def test_noise_estimate_matches_oracle(cfg, tol):
    api = _api()
    cube = synth.config_cube(cfg, keep_clean=False)
    say("noise cfg", cfg, cube.Y.shape)
    Y = torch.tensor(cube.Y, device="cuda")
    sigma, st = api.estimate_noise(Y)
    ref = O.noise_estimate(cube.Y.reshape(-1, cube.Y.shape[2]).astype(np.float64))
    assert int(st.cpu()[0]) == 0
    assert np.abs(sigma.cpu().numpy() / ref - 1).max() <= tol


def test_subspace_matches_oracle():
    api = _api()
    cube = synth.config_cube(1, keep_clean=False)
    Y = torch.tensor(cube.Y, device="cuda")
    ref = O.hyres(cube.Y, 4, 3)
    V, ev, st = api.subspace(Y, 4, torch.tensor(ref["sigma"], device="cuda"))
    assert int(st.cpu()[0]) == 0
    np.testing.assert_allclose(ev.cpu().numpy(), ref["evals"], rtol=1e-11, atol=1e-11 * ref["evals"][0])
    np.testing.assert_allclose(V.cpu().numpy(), ref["V"], atol=1e-9)


# ------------------------------------------------------------- end to end
def _check_denoise(Y, r, L, tol, sigma=None, lam=None, name="", precision="native", scope="all",
                   rank_rule=None):
    api = _api()
    say("denoise", name, Y.shape, Y.dtype, "r", r, "L", L, precision, scope, rank_rule)
    Yt = torch.tensor(Y, device="cuda")
    X, info = api.denoise(Yt, r, L, precision=precision,
                          sigma=None if sigma is None else torch.tensor(sigma),
                          lam=None if lam is None else torch.tensor(lam), scope=scope, rank_rule=rank_rule)
    X = X.cpu().numpy()
    st = int(info["status"].cpu()[0])
    assert st & ~8 == 0, st
    det = scope == "detail"
    ref = O.hyres(Y.astype(np.float64), r, L, sigma=sigma, lam=lam, detail_only=det, rank_rule=rank_rule)
    if rank_rule is not None:
        # the device's choice is the oracle's; the components beyond it are zero
        k = int(info["rank"].cpu()[0])
        say("   rank", rank_rule, "device", k, "oracle", ref["rank"])
        assert k == ref["rank"], (k, ref["rank"])
        assert not info["V"][:, k:].any()
        r = k
    lam_g = info["lam"].cpu().numpy()[:r]
    if lam is None:
        eps = SP.EPS["mixed" if precision == "mixed" else Y.dtype.name]
        other = False
        for i in range(r):
            if abs(lam_g[i] - ref["lam"][i]) > 1e-4 * max(ref["lam"][i], 1e-3):
                # a different near-optimal candidate: check its oracle risk, then compare at it
                bi = ref["B"][i]
                if det:
                    hL, wL = O.level_shapes(Y.shape[0], Y.shape[1], L)[-1]
                    bi = bi[: bi.size - hL * wL]
                ok, gap, allowed = SP.accept(bi, lam_g[i], ref["lam"][i], ref["sure"][i], eps)
                say("   component", i, "device lambda", lam_g[i], "oracle", ref["lam"][i], "SURE gap", gap,
                    "allowed", allowed)
                assert ok, (i, lam_g[i], ref["lam"][i], gap, allowed)
                other = True
        # the SURE candidate set of the detail scope excludes LL_L
        if other:
            ref = O.hyres(Y.astype(np.float64), r, L, sigma=sigma, lam=lam_g, detail_only=det)
            ref["rank"] = r
    e, emax = PM.errors(X, ref["X"])
    say("   rel err", e, "max err / max", emax, "lam gpu", lam_g, "lam ref", ref["lam"])
    PM.assert_close(X, ref["X"], tol, name)
    np.testing.assert_allclose(info["sigma"].cpu().numpy(), ref["sigma"], rtol=max(tol * 10, 1e-12))
    return X, info, ref


def test_denoise_config1_fp64():
    cube = synth.config_cube(1, keep_clean=False)
    _check_denoise(cube.Y, 4, 3, 1e-10, name="c1")


@pytest.mark.parametrize("H,W,p,r,L", [(97, 133, 40, 5, 3), (64, 200, 17, 1, 2), (33, 40, 2, 2, 2),
                                       (128, 128, 100, 12, 4)])
def test_denoise_ragged_fp64_and_fp32(H, W, p, r, L):
    cube = synth.mixing_cube(H * W + p, H, W, p, min(r, 6), 12.0, L, dtype=np.float64, keep_clean=False)
    # clipped spectra can leave a band with no signal and therefore no noise;
    # a small independent floor keeps every band's regression well posed
    Y = cube.Y + 1e-3 * np.random.default_rng(H + W).standard_normal(cube.Y.shape)
    _check_denoise(Y, r, L, 1e-10, name="ragged64")
    _check_denoise(Y.astype(np.float32), r, L, 1e-5, name="ragged32")


def test_denoise_given_sigma_and_lambda():
    cube = synth.config_cube(1, keep_clean=False)
    sig = cube.sigma_true
    lam = np.array([0.5, 1.0, 1.5, 2.0])
    _check_denoise(cube.Y, 4, 3, 1e-10, sigma=sig, lam=lam, name="given")
    _check_denoise(cube.Y.astype(np.float32), 4, 3, 1e-5, sigma=sig, lam=lam, name="given32")


def test_denoise_config2_fp32_full_size():
    cube = synth.config_cube(2, keep_clean=False)
    _check_denoise(cube.Y, 8, 4, 1e-5, name="c2")


def test_denoise_config2_mixed_full_size():
    cube = synth.config_cube(2, keep_clean=False)
    X, info, ref = _check_denoise(cube.Y, 8, 4, 1e-3, name="c2-mixed", precision="mixed")
    # the FP32 refinement: Ritz values and the basis at FP32 accuracy
    ev = info["evals"].cpu().numpy()[:8]
    e_ev = float(np.max(np.abs(ev / ref["evals"][:8] - 1)))
    V = info["V"].cpu().numpy()
    cosines = np.linalg.svd(V.T @ ref["V"], compute_uv=False)
    e_v = float(np.max(np.abs(V - ref["V"])))
    say("   mixed evals rel err", e_ev, "V max abs diff", e_v, "min cosine", cosines.min())
    assert e_ev <= 1e-5
    assert e_v <= 1e-3


def test_denoise_mixed_largest_rank():
    """Rank 16, the largest (16 sources, so the subspace is well separated):
    the rotated first analysis level then holds 16 component windows per block,
    more than 64 KB of LDS."""
    cube = synth.mixing_cube(7016, 70, 150, 48, 16, 15.0, 2, dtype=np.float32, keep_clean=False)
    _check_denoise(cube.Y, 16, 2, 1e-3, name="mixed-r16", precision="mixed")


@pytest.mark.parametrize("H,W,p,r,L", [(97, 133, 40, 5, 3), (128, 128, 100, 12, 4), (64, 96, 191, 6, 3)])
def test_denoise_mixed_ragged(H, W, p, r, L):
    cube = synth.mixing_cube(H * W + p, H, W, p, min(r, 6), 12.0, L, dtype=np.float32, keep_clean=False)
    Y = cube.Y + np.float32(1e-3) * np.random.default_rng(H + W).standard_normal(cube.Y.shape).astype(np.float32)
    _check_denoise(Y, r, L, 1e-3, name="mixed", precision="mixed")


def test_denoise_detail_scope_matches_oracle():
    # one threshold per component over the detail coefficients only; LL_L kept
    cube = synth.config_cube(1, keep_clean=False)
    _check_denoise(cube.Y, 4, 3, 1e-10, name="c1-detail", scope="detail")
    c = synth.mixing_cube(977, 97, 133, 40, 5, 12.0, 3, dtype=np.float64, keep_clean=False)
    Y = c.Y + 1e-3 * np.random.default_rng(5).standard_normal(c.Y.shape)
    _check_denoise(Y.astype(np.float32), 5, 3, 1e-5, name="ragged32-detail", scope="detail")
    _check_denoise(Y.astype(np.float32), 5, 3, 1e-3, name="ragged-mixed-detail", scope="detail",
                   precision="mixed")


def test_denoise_fp32_native_224_bands_matches_oracle():
    # the widest band count: three-part native Gram (14 band tiles) and the
    # largest register tiling of the small solve
    c = synth.mixing_cube(224, 128, 160, 224, 6, 10.0, 4, dtype=np.float64, keep_clean=False)
    Y = (c.Y + 1e-3 * np.random.default_rng(224).standard_normal(c.Y.shape)).astype(np.float32)
    _check_denoise(Y, 10, 4, 1e-5, name="p224-native")
    _check_denoise(Y, 10, 4, 1e-3, name="p224-mixed", precision="mixed")


@pytest.mark.parametrize("rule", ["hysime", "sure"])
def test_denoise_with_data_chosen_rank(rule):
    """The rank chosen on the device (HySime, or SURE of the truncated whitened
    cube) equals the oracle's, and the solve at that rank matches: the
    64 x 64 x 32 FP64 cube and the 349 x 1905 x 144 FP32 cube, largest rank 8."""
    cube = synth.config_cube(1, keep_clean=False)
    _check_denoise(cube.Y, 8, 3, 1e-10, name="c1-" + rule, rank_rule=rule)
    cube = synth.config_cube(2, keep_clean=False)
    _check_denoise(cube.Y, 8, 4, 1e-5, name="c2-" + rule, rank_rule=rule)


@pytest.mark.parametrize("case", ["fp64", "fp32", "mixed-224", "sure-rank"])
def test_eigensolve_diagnostics(case):
    """The eigensolve's own accuracy report: ||C V - V Lambda|| / ||C|| and
    max |V^T V - I| over the eigenpairs used, on the device, at FP64 rounding
    level; the host recomputes the residual of the returned pairs on the FP64
    Gram of the cube (FP32 cubes: at the level of the device's FP32 chunk sums;
    the mixed path returns the FP32 Rayleigh-Ritz pairs)."""
    api = _api()
    if case == "mixed-224":
        c = synth.mixing_cube(224, 96, 80, 224, 6, 12.0, 3, dtype=np.float32, keep_clean=False)
        Y = c.Y + np.float32(1e-3) * np.random.default_rng(224).standard_normal(c.Y.shape).astype(np.float32)
        r, L, prec, rule = 10, 3, "mixed", None
    else:
        c = synth.mixing_cube(97, 97, 133, 40, 5, 12.0, 3, dtype=np.float64, keep_clean=False)
        Y = c.Y + 1e-3 * np.random.default_rng(7).standard_normal(c.Y.shape)
        Y = Y.astype(np.float32) if case == "fp32" else Y
        r, L, prec, rule = 8, 3, "native", ("sure" if case == "sure-rank" else None)
    say("eig diagnostics", case, Y.shape, Y.dtype, "r", r)
    X, info = api.denoise(torch.tensor(Y, device="cuda"), r, L, precision=prec, rank_rule=rule, check_eigs=True)
    resid, orth = float(info["eig_resid"].item()), float(info["eig_orth"].item())
    k = int(info["rank"].item())
    Yd = Y.astype(np.float64).reshape(-1, Y.shape[2])
    s = info["sigma"].cpu().numpy()
    Cm = (Yd.T @ Yd) / np.outer(s, s)
    V = info["V"].cpu().numpy()[:, :k]
    ev = info["evals"].cpu().numpy()[:k]
    host = float(np.linalg.norm(Cm @ V - V * ev) / np.linalg.norm(Cm))
    say("   rank", k, "device resid", resid, "orth", orth, "host resid of the returned pairs", host)
    assert 0 < k <= r
    assert resid <= 1e-13 and orth <= 1e-13
    # FP32 cubes: the device Gram sums 64-pixel chunks in FP32 before FP64, so
    # its exact eigenpairs sit that far from those of the FP64 Gram
    assert host <= (1e-5 if prec == "mixed" else 1e-6 if Y.dtype == np.float32 else 1e-12)


def test_denoise_is_deterministic():
    api = _api()
    cube = synth.config_cube(1, keep_clean=False)
    Y = torch.tensor(cube.Y.astype(np.float32), device="cuda")
    a, _ = api.denoise(Y, 4, 3)
    b, _ = api.denoise(Y, 4, 3)
    assert torch.equal(a, b)


def test_noise_flags_nonfinite_and_dependent_bands():
    api = _api()
    cube = synth.config_cube(1, keep_clean=False)
    Y = cube.Y.copy()
    Y[3, 4, 5] = np.nan
    _, info = api.denoise(torch.tensor(Y, device="cuda"), 4, 3)
    assert int(info["status"].cpu()[0]) & 2
    Y = cube.Y.copy()
    Y[:, :, 7] = Y[:, :, 3]                       # a duplicated band: the Gram is singular
    _, info = api.denoise(torch.tensor(Y, device="cuda"), 4, 3)
    assert int(info["status"].cpu()[0]) & 1


@pytest.mark.parametrize("side_stream", [False, True])
def test_stage_timers_time_every_stage(side_stream):
    """The stage timers record every stage of a solve, on torch's default (null)
    stream as on a stream of its own."""
    import ctypes as C
    from paper_2204_06979_amd import _lib as L
    api = _api()
    lib = L.lib()
    cube = synth.mixing_cube(7, 96, 80, 40, 4, 12.0, 3, dtype=np.float32, keep_clean=False)
    Yt = torch.tensor(cube.Y, device="cuda")
    h = api._handle(Yt.device)
    s = torch.cuda.Stream() if side_stream else torch.cuda.default_stream()
    nst = 7
    lib.hyres_profile_enable(h, (1 << nst) - 1)
    try:
        with torch.cuda.stream(s):
            api.denoise(Yt, 4, 3)
            api.denoise(Yt, 4, 3)
        torch.cuda.synchronize()
        ms = (C.c_double * nst)()
        cnt = (C.c_int * nst)()
        L.check(lib.hyres_profile_read(h, ms, cnt), "profile read")
    finally:
        lib.hyres_profile_enable(h, 0)
    say("stage ms", list(ms), "counts", list(cnt))
    assert list(cnt) == [2] * nst
    assert all(m > 0.0 for m in ms)
