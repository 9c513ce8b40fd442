"""Plain FP64 CPU oracle of HyMiNoR's sparse-noise stage (test infrastructure only).

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this module; it shares no code with the GPU library.

Section 2.1 describes HyMiNoR as HyRes followed by the removal of the sparse
noise that HyRes leaves, by an l1-l1 problem solved with a (modified) split
Bregman method; the paper prints neither the problem nor the iteration.  The
reading taken here (listed with the other readings in the design notes):

  S1  the input H is the HyRes output, one spectrum h (p bands) per pixel;
  S2  per pixel, x = argmin_x ||h - x||_1 + lam ||D x||_1, D the (p-1) x p
      first-order spectral difference (D x)_i = x_{i+1} - x_i: an l1 data term
      that lets a few bands move far (sparse noise) and an l1 spectral
      roughness term that keeps spectral edges;
  S3  split Bregman with s = h - x and u = D x, penalties mu1 and mu2, all
      auxiliary and Bregman variables starting at zero:
        x  <- (mu1 I + mu2 D^T D)^-1 (mu1 (h - s + b1) + mu2 D^T (u - b2))
        s  <- soft(h - x + b1, 1 / mu1)
        u  <- soft(D x + b2, lam / mu2)
        b1 <- b1 + h - x - s
        b2 <- b2 + D x - u
      for a fixed number of sweeps K >= 1; the result is the x of sweep K.

The x step is the exact solution of the tridiagonal system (a dense solve
here); nothing is truncated or reordered.
"""
from __future__ import annotations

from typing import Dict, Optional

import numpy as np

from oracle import hyres_oracle as HO

__all__ = ["spectral_difference", "l1l1_objective", "l1l1_split_bregman", "hyminor"]


def spectral_difference(p: int) -> np.ndarray:
    """(p-1) x p first-order difference along the bands: (D x)_i = x_{i+1} - x_i."""
    D = np.zeros((max(p - 1, 0), p))
    for i in range(p - 1):
        D[i, i] = -1.0
        D[i, i + 1] = 1.0
    return D


def l1l1_objective(h: np.ndarray, x: np.ndarray, lam: float) -> np.ndarray:
    """||h - x||_1 + lam ||D x||_1 per pixel (last axis = bands)."""
    return np.abs(h - x).sum(-1) + lam * np.abs(np.diff(x, axis=-1)).sum(-1)


def _soft(v: np.ndarray, t: float) -> np.ndarray:
    return np.sign(v) * np.maximum(np.abs(v) - t, 0.0)


def l1l1_split_bregman(Hc: np.ndarray, lam: float, mu1: float, mu2: float, iters: int) -> np.ndarray:
    """S2-S3 on every pixel of Hc (... x p, any leading shape), in FP64."""
    if iters < 1 or not (mu1 > 0 and mu2 > 0 and lam >= 0):
        raise ValueError("need iters >= 1, mu1 > 0, mu2 > 0, lam >= 0")
    shape = Hc.shape
    p = shape[-1]
    h = np.asarray(Hc, dtype=np.float64).reshape(-1, p)
    D = spectral_difference(p)
    M = mu1 * np.eye(p) + mu2 * D.T @ D
    s = np.zeros_like(h)
    b1 = np.zeros_like(h)
    u = np.zeros((h.shape[0], p - 1))
    b2 = np.zeros_like(u)
    x = h
    for _ in range(iters):
        rhs = mu1 * (h - s + b1) + mu2 * (u - b2) @ D
        x = np.linalg.solve(M, rhs.T).T
        Dx = x @ D.T
        s = _soft(h - x + b1, 1.0 / mu1)
        u = _soft(Dx + b2, lam / mu2)
        b1 = b1 + h - x - s
        b2 = b2 + Dx - u
    return x.reshape(shape)


def hyminor(Y: np.ndarray, r: int, L: int, lam: float, mu1: float, mu2: float, iters: int,
            sigma: Optional[np.ndarray] = None, hyres_lam: Optional[np.ndarray] = None,
            rank_rule: Optional[str] = None) -> Dict[str, np.ndarray]:
    """HyRes (S1), then the l1-l1 sparse-noise stage on its output."""
    res = HO.hyres(Y, r, L, sigma=sigma, lam=hyres_lam, rank_rule=rank_rule)
    out = dict(res)
    out["X_hyres"] = res["X"]
    out["X"] = l1l1_split_bregman(res["X"], lam, mu1, mu2, iters)
    return out
