"""Pins of the WSRRR oracle: the polar factor against scipy's polar
decomposition and as the maximiser of tr(V^T M) over orthonormal V; the
objective never increasing over the alternating steps (even sizes, where the
transform is orthogonal); the fixed point without thresholds (the top-r
eigenvectors: X is then the PCA truncation); symmetry of V^T Yw^T W F at a
fixed point (the first-order condition of the Procrustes step); and K = 0
reducing to HyRes."""
import numpy as np
import pytest
from scipy import linalg

from oracle import hyres_oracle as O
from oracle import wsrrr_oracle as WS
from paper_2204_06979_amd import synth


def test_polar_factor_against_scipy_and_optimality():
    rng = np.random.default_rng(1)
    M = rng.standard_normal((12, 4))
    V = WS.polar_factor(M)
    U, _ = linalg.polar(M)                       # M = U P, U with orthonormal columns
    np.testing.assert_allclose(V, U, atol=1e-12)
    np.testing.assert_allclose(V.T @ V, np.eye(4), atol=1e-12)
    best = np.trace(V.T @ M)
    for _ in range(200):
        Qr, _ = np.linalg.qr(rng.standard_normal((12, 4)))
        assert np.trace(Qr.T @ M) <= best + 1e-12
        Vp, _ = np.linalg.qr(V + 1e-3 * rng.standard_normal((12, 4)))
        assert np.trace(Vp.T @ M) <= best + 1e-12


def test_objective_never_increases():
    cube = synth.mixing_cube(41, 64, 48, 24, 3, 10.0, 3, dtype=np.float64, keep_clean=False)
    out = WS.wsrrr(cube.Y, 4, 3, 6, history=True)
    J = out["objective"]
    assert np.all(np.diff(J) <= 1e-9 * J[0]), J
    assert J[-1] < J[0]


def test_without_thresholds_the_eigenvectors_are_a_fixed_point():
    rng = np.random.default_rng(2)
    Y = rng.standard_normal((32, 40, 10)) + np.linspace(0, 2, 10)
    out = WS.wsrrr(Y, 3, 2, 4, lam=np.zeros(3))
    ref = O.hyres(Y, 3, 2, lam=np.zeros(3))
    np.testing.assert_allclose(np.abs(out["V"].T @ ref["V"]), np.eye(3), atol=1e-9)
    sig = ref["sigma"]
    Yw = Y.reshape(-1, 10) / sig
    pca = (Yw @ ref["V"] @ ref["V"].T * sig).reshape(Y.shape)
    np.testing.assert_allclose(out["X"], pca, atol=1e-9)


def test_first_order_condition_at_convergence():
    cube = synth.mixing_cube(43, 32, 32, 16, 3, 15.0, 2, dtype=np.float64, keep_clean=False)
    out = WS.wsrrr(cube.Y, 3, 2, 200)     # the alternation converges linearly
    Yw = cube.Y.reshape(-1, 16) / out["sigma"]
    V = out["V"]
    Zh = (out["X"].reshape(-1, 16) / out["sigma"]) @ V          # W F, since V^T V = I
    S = V.T @ (Yw.T @ Zh)
    np.testing.assert_allclose(S, S.T, atol=1e-7 * np.abs(S).max())


def test_zero_iterations_is_hyres():
    cube = synth.config_cube(1, keep_clean=False)
    out = WS.wsrrr(cube.Y, 4, 3, 0)
    np.testing.assert_allclose(out["X"], out["hyres_X"], rtol=0, atol=1e-12)


def test_a_zero_component_keeps_its_direction():
    rng = np.random.default_rng(6)
    Vp, _ = np.linalg.qr(rng.standard_normal((9, 3)))
    M = rng.standard_normal((9, 3))
    M[:, 1] = 0.0
    V = WS.procrustes_step(M, Vp)
    np.testing.assert_allclose(V.T @ V, np.eye(3), atol=1e-12)
    np.testing.assert_allclose(V[:, [0, 2]], WS.polar_factor(M[:, [0, 2]]), atol=1e-12)
    # column 1: the previous direction with its parts along the other two removed
    v = Vp[:, 1] - V[:, [0, 2]] @ (V[:, [0, 2]].T @ Vp[:, 1])
    np.testing.assert_allclose(V[:, 1], v / np.linalg.norm(v), atol=1e-12)
    # nothing zero: the plain polar factor
    M2 = rng.standard_normal((9, 3))
    np.testing.assert_allclose(WS.procrustes_step(M2, Vp), WS.polar_factor(M2), atol=1e-12)
