"""Plain FP64 CPU oracle of FORPDN (test infrastructure only).

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this module; it shares no code with the GPU library.

Section 2.1 lists FORPDN (first-order spectral roughness penalty denoising)
as a full-rank, wavelet-based method aimed at additive Gaussian noise, and
prints nothing more.  The reading taken here (listed with the other readings
in the design notes):

  F1  per-band noise sigma by the same regression estimator as HyRes (O2);
      the cube is whitened band by band (Y / sigma);
  F2  every whitened band is transformed by the same L-level periodised 2-D
      db2 transform as HyRes uses (O6); the coefficients of one position form
      a p-vector across the bands;
  F3  the coefficient vectors are split into L + 1 groups: the three detail
      subbands of each level, and the coarsest approximation;
  F4  in group j every coefficient vector c becomes the penalised least-
      squares estimate argmin_x ||c - x||^2 + lam_j ||D x||^2, D the first-
      order spectral difference, i.e. x = (I + lam_j D^T D)^-1 c (full rank:
      no subspace);
  F5  lam_j minimises Stein's unbiased risk estimate of that linear smoother
      at unit noise, SURE(lam) = ||C - C S||^2 - N p + 2 N tr(S) with
      S = (I + lam D^T D)^-1 and C the N x p coefficient matrix of the group,
      over the grid lam = 10^(k/10), k = -40..40 (the smallest lam on ties);
  F6  inverse transform of every band, then un-whitening (X * sigma).
"""
from __future__ import annotations

from typing import Dict, List, Optional, Tuple

import numpy as np

from oracle import hyres_oracle as HO

__all__ = ["LAM_GRID", "roughness_smoother", "smoother_sure", "group_slices", "forpdn"]

LAM_GRID = np.array([10.0 ** (k / 10.0) for k in range(-40, 41)])


def _difference(p: int) -> np.ndarray:
    D = np.zeros((max(p - 1, 0), p))
    for i in range(p - 1):
        D[i, i] = -1.0
        D[i, i + 1] = 1.0
    return D


def roughness_smoother(p: int, lam: float) -> np.ndarray:
    """S = (I + lam D^T D)^-1, p x p (F4)."""
    D = _difference(p)
    return np.linalg.inv(np.eye(p) + lam * D.T @ D)


def smoother_sure(C: np.ndarray, lam: float) -> float:
    """F5 at one lam: ||C - C S||^2 - N p + 2 N tr(S), unit noise, C is N x p."""
    N, p = C.shape
    S = roughness_smoother(p, lam)
    R = C - C @ S
    return float(np.sum(R * R) - N * p + 2.0 * N * np.trace(S))


def group_slices(H: int, W: int, L: int) -> List[Tuple[int, int]]:
    """F3: [start, stop) of each group in a coefficient vector of dwt2 (levels 1..L, then LL_L)."""
    out = []
    o = 0
    for h, w in HO.level_shapes(H, W, L):
        out.append((o, o + 3 * h * w))
        o += 3 * h * w
    out.append((o, HO.coeff_count(H, W, L)))
    return out


def forpdn(Y: np.ndarray, L: int, sigma: Optional[np.ndarray] = None,
           lam: Optional[np.ndarray] = None) -> Dict[str, np.ndarray]:
    """F1-F6 on an H x W x p cube in FP64.  ``sigma`` and ``lam`` (one per
    group) may be given.  Returns X, sigma, lam, sure (minimum per group)."""
    Y = np.asarray(Y, dtype=np.float64)
    H, W, p = Y.shape
    Y2 = Y.reshape(H * W, p)
    if sigma is None:
        sigma = HO.noise_estimate(Y2)                               # F1
    sigma = np.asarray(sigma, dtype=np.float64)
    Yw = Y / sigma[None, None, :]
    B = np.stack([HO.dwt2(Yw[:, :, b], L) for b in range(p)])       # F2: p x Nc
    groups = group_slices(H, W, L)                                  # F3
    lam_out = np.empty(len(groups))
    sure_out = np.empty(len(groups))
    for j, (a, b) in enumerate(groups):
        C = B[:, a:b].T                                             # N_j x p
        if lam is None:
            vals = [smoother_sure(C, t) for t in LAM_GRID]          # F5
            k = int(np.argmin(vals))
            lj, sj = float(LAM_GRID[k]), float(vals[k])
        else:
            lj = float(lam[j])
            sj = smoother_sure(C, lj)
        lam_out[j] = lj
        sure_out[j] = sj
        B[:, a:b] = (C @ roughness_smoother(p, lj)).T               # F4 (S is symmetric)
    Xw = np.stack([HO.idwt2(B[b], H, W, L) for b in range(p)], axis=2)   # F6
    return dict(X=Xw * sigma[None, None, :], sigma=sigma, lam=lam_out, sure=sure_out)
