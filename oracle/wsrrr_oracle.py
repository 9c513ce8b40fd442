"""Plain FP64 CPU oracle of WSRRR (test infrastructure only).

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this module; it shares no code with the GPU library.

Section 2.1 lists WSRRR (wavelet-based sparse reduced-rank regression) as a
low-rank, wavelet-based method for Gaussian noise that can also extract
features, and prints nothing more.  The reading taken here (listed with the
other readings in the design notes), in the whitened frame of HyRes
(Yw = Y / sigma, unit noise):

  W1  model Yw = W F V^T + noise: F the wavelet coefficients of r component
      images (W the synthesis of the HyRes transform), V a p x r matrix with
      orthonormal columns; the estimate minimises
        J(F, V) = 1/2 ||Yw - W F V^T||^2 + sum_i lam_i ||f_i||_1,  V^T V = I;
  W2  start: HyRes (its sigma, its subspace V_0, its SURE thresholds lam_i,
      which stay fixed, and its F_0);
  W3  alternate K times:
        V <- the orthonormal factor of the polar decomposition of Yw^T W F
             (the maximiser of tr(V^T Yw^T W F) over V^T V = I: Procrustes);
             a component whose coefficients are all zero (the SURE threshold
             can zero a whole component) does not enter the objective, so
             its column is free: it keeps its previous direction, made
             orthonormal to the other columns (Gram-Schmidt, in index order);
        F <- soft(W^T Yw V, lam)          (the F step of HyRes with the new V);
  W4  X = (W F V^T) * sigma.
For even image sizes W is orthogonal and each half-step does not increase J.
"""
from __future__ import annotations

from typing import Dict, Optional

import numpy as np

from oracle import hyres_oracle as HO

__all__ = ["polar_factor", "procrustes_step", "objective", "wsrrr"]


def polar_factor(M: np.ndarray) -> np.ndarray:
    """Orthonormal factor of M (p x r, full column rank): U Q^T for M = U S Q^T."""
    U, _, Qt = np.linalg.svd(M, full_matrices=False)
    return U @ Qt


def procrustes_step(M: np.ndarray, V_prev: np.ndarray) -> np.ndarray:
    """W3's V step: the polar factor of the columns of M that are not zero
    (squared norm above 1e-24 of the largest); each zero column takes the
    previous direction, orthonormalised against the columns already set."""
    nrm = np.sum(M * M, axis=0)
    live = nrm > 1e-24 * nrm.max()
    V = np.zeros_like(V_prev)
    V[:, live] = polar_factor(M[:, live])
    for k in np.flatnonzero(~live):
        v = V_prev[:, k].copy()
        for j in range(V.shape[1]):
            if live[j] or j < k:
                v -= (V[:, j] @ v) * V[:, j]
        V[:, k] = v / np.linalg.norm(v)
    return V


def _f_step(Yw: np.ndarray, V: np.ndarray, lam: np.ndarray, H: int, W: int, L: int):
    """F = soft(W^T Yw V, lam) per component; returns (F rows, W F as n x r)."""
    n = H * W
    Z = Yw @ V
    r = V.shape[1]
    F = np.stack([HO.soft_threshold(HO.dwt2(Z[:, i].reshape(H, W), L), lam[i]) for i in range(r)])
    Zh = np.stack([HO.idwt2(F[i], H, W, L).reshape(n) for i in range(r)], axis=1)
    return F, Zh


def objective(Yw: np.ndarray, F: np.ndarray, Zh: np.ndarray, V: np.ndarray, lam: np.ndarray) -> float:
    """J of W1 (Zh = W F as n x r)."""
    R = Yw - Zh @ V.T
    return float(0.5 * np.sum(R * R) + np.sum(lam * np.abs(F).sum(axis=1)))


def wsrrr(Y: np.ndarray, r: int, L: int, iters: int, sigma: Optional[np.ndarray] = None,
          lam: Optional[np.ndarray] = None, history: bool = False) -> Dict[str, np.ndarray]:
    """W1-W4 on an H x W x p cube in FP64."""
    Y = np.asarray(Y, dtype=np.float64)
    H, Wd, p = Y.shape
    base = HO.hyres(Y, r, L, sigma=sigma, lam=lam)                     # W2
    sig = base["sigma"]
    lam_ = base["lam"]
    Yw = Y.reshape(H * Wd, p) / sig[None, :]
    V = base["V"]
    F, Zh = _f_step(Yw, V, lam_, H, Wd, L)
    hist = [objective(Yw, F, Zh, V, lam_)]
    for _ in range(iters):                                             # W3
        V = procrustes_step(Yw.T @ Zh, V)
        if history:
            hist.append(objective(Yw, F, Zh, V, lam_))
        F, Zh = _f_step(Yw, V, lam_, H, Wd, L)
        if history:
            hist.append(objective(Yw, F, Zh, V, lam_))
    X = (Zh @ V.T * sig[None, :]).reshape(H, Wd, p)                     # W4
    out = dict(X=X, sigma=sig, V=V, lam=lam_, hyres_X=base["X"])
    if history:
        out["objective"] = np.array(hist)
    return out
