"""Pins of the FORPDN oracle against facts that do not come from the oracle:
the closed-form 2-band smoother, numerical minimisation of the penalised
least-squares objective, the lam -> 0 and lam -> infinity limits, the
diagonalisation of D^T D by the DCT-II basis (the eigenpairs are textbook)
giving SURE in closed form, Monte-Carlo unbiasedness of SURE, the group
partition of the coefficient vector, exact reconstruction when nothing is
smoothed, the band mean when everything is, and the effect on a noisy cube."""
import math

import numpy as np
import pytest
from scipy import optimize

from oracle import forpdn_oracle as F
from oracle import hyres_oracle as O
from paper_2204_06979_amd import synth


def test_two_band_smoother_closed_form():
    for lam in [0.1, 1.0, 7.5]:
        want = np.array([[1 + lam, lam], [lam, 1 + lam]]) / (1 + 2 * lam)
        np.testing.assert_allclose(F.roughness_smoother(2, lam), want, rtol=1e-14, atol=1e-15)


@pytest.mark.parametrize("lam", [0.05, 0.8, 12.0])
def test_smoother_minimises_the_penalised_objective(lam):
    rng = np.random.default_rng(2)
    c = rng.standard_normal(9)
    obj = lambda x: np.sum((c - x) ** 2) + lam * np.sum(np.diff(x) ** 2)     # noqa: E731
    res = optimize.minimize(obj, c, method="BFGS", options={"gtol": 1e-12})
    np.testing.assert_allclose(F.roughness_smoother(9, lam) @ c, res.x, atol=1e-6)


def test_limits_of_the_smoother():
    p = 11
    np.testing.assert_allclose(F.roughness_smoother(p, 1e-12), np.eye(p), atol=1e-10)
    np.testing.assert_allclose(F.roughness_smoother(p, 1e9), np.full((p, p), 1.0 / p), atol=1e-6)


@pytest.mark.parametrize("p", [2, 7, 32])
def test_sure_in_the_dct_basis(p):
    # D^T D (first-order differences, free ends) has eigenvalues 2 - 2 cos(pi k / p)
    # with the DCT-II vectors cos(pi k (i + 1/2) / p): SURE is then diagonal
    i = np.arange(p)
    Q = np.stack([np.cos(math.pi * k * (i + 0.5) / p) for k in range(p)], axis=1)
    Q /= np.linalg.norm(Q, axis=0)
    d = 2.0 - 2.0 * np.cos(math.pi * np.arange(p) / p)
    Dm = np.diff(np.eye(p), axis=0)
    np.testing.assert_allclose(Dm.T @ Dm @ Q, Q * d, atol=1e-12)
    rng = np.random.default_rng(p)
    C = rng.standard_normal((50, p)) + np.linspace(0, 3, p)
    e = np.sum((C @ Q) ** 2, axis=0)
    for lam in [0.01, 0.3, 5.0, 200.0]:
        f = 1.0 / (1.0 + lam * d)
        closed = np.sum(e * (1 - f) ** 2) - C.size + 2 * C.shape[0] * np.sum(f)
        assert abs(F.smoother_sure(C, lam) - closed) <= 1e-9 * max(1.0, abs(closed))


def test_sure_is_unbiased_monte_carlo():
    rng = np.random.default_rng(9)
    N, p, lam = 40, 12, 2.0
    theta = np.cumsum(rng.standard_normal((N, p)), axis=1) * 0.3
    S = F.roughness_smoother(p, lam)
    sure, risk = [], []
    for _ in range(3000):
        C = theta + rng.standard_normal((N, p))
        sure.append(F.smoother_sure(C, lam))
        risk.append(np.sum((C @ S - theta) ** 2))
    sure, risk = np.array(sure), np.array(risk)
    se = np.std(sure - risk) / math.sqrt(len(sure))
    assert abs(sure.mean() - risk.mean()) < 4 * se + 1e-9


def test_group_slices_partition_the_coefficients():
    for H, W, L in [(64, 64, 3), (37, 53, 3), (349, 191, 4)]:
        g = F.group_slices(H, W, L)
        assert g[0][0] == 0 and g[-1][1] == O.coeff_count(H, W, L)
        assert all(g[k][1] == g[k + 1][0] for k in range(len(g) - 1))
        assert len(g) == L + 1
        hL, wL = O.level_shapes(H, W, L)[-1]
        assert g[-1][1] - g[-1][0] == hL * wL


@pytest.mark.parametrize("H,W", [(32, 40), (33, 27)])
def test_nothing_smoothed_reconstructs_the_cube(H, W):
    rng = np.random.default_rng(H)
    Y = rng.standard_normal((H, W, 9)) + 3.0
    out = F.forpdn(Y, 3, lam=np.full(4, 1e-13))
    np.testing.assert_allclose(out["X"], Y, atol=1e-9)


def test_everything_smoothed_gives_the_whitened_band_mean():
    rng = np.random.default_rng(4)
    Y = rng.standard_normal((16, 24, 6)) + np.arange(6)
    sig = np.array([1.0, 2.0, 0.5, 1.5, 1.0, 3.0])
    out = F.forpdn(Y, 2, sigma=sig, lam=np.full(3, 1e10))
    want = (Y / sig).mean(axis=2, keepdims=True) * sig
    np.testing.assert_allclose(out["X"], want, atol=1e-6)


def test_denoises_smooth_spectra():
    cube = synth.mixing_cube(12, 64, 64, 48, 4, 10.0, 3, dtype=np.float64, keep_clean=True)
    out = F.forpdn(cube.Y, 3)
    e_noisy = np.linalg.norm(cube.Y - cube.X)
    e_f = np.linalg.norm(out["X"] - cube.X)
    assert e_f < 0.6 * e_noisy, (e_f, e_noisy)
    # SURE picks a finer penalty for the approximation than for the finest details
    assert out["lam"][-1] <= out["lam"][0]
    assert np.all(np.isin(out["lam"], F.LAM_GRID))
