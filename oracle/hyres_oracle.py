"""Plain FP64 CPU oracle of the HyRes denoiser (test infrastructure only).

This module is the reference that the HIP path is checked against.  It is
slow on purpose and shares no code with the GPU library: only the test suite,
the smoke check and the benchmark's CPU-baseline leg may import it.

The paper (Section 2.1) names HyRes as a low-rank, wavelet-based, parameter-
free Gaussian denoiser and cites the original method; it prints no equations.
The steps below are the method as it is commonly stated for that family and
as the spec path lists it:

  O1  Y (H x W x p) -> n x p matrix, row = y*W + x.
  O2  per-band noise: regress band i on the other p-1 bands (no intercept);
      sigma_i^2 = residual sum of squares / n.
  O3  whitening: Yw = Y / sigma (per band).
  O4  subspace: C = Yw^T Yw; eigenvectors sorted by descending eigenvalue;
      V = first r; sign rule: the entry of largest magnitude is positive
      (first such index on ties).
  O5  projection: Z = Yw V; component images Z_i (H x W).
  O6  L-level periodised 2-D Daubechies 4-tap (db2) transform per component.
  O7  per-component threshold: exact minimiser of Stein's unbiased risk
      estimate of soft thresholding at unit noise over {0} U {|b_k|}.
  O8  soft threshold.
  O9  inverse transform.
  O10 back-projection: Xhat = (sum_i Zhat_i v_i^T) * sigma.

Readings where the paper is silent are listed in the design notes of the
repository; the ones that change numbers are: no intercept and divisor n in
O2, uncentred Gram in O4, odd lengths extended by repeating the last sample
in O6, every coefficient of a component (including the coarsest
approximation) thresholded with one threshold in O7.
"""
from __future__ import annotations

import math
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

__all__ = [
    "DB2", "HAAR", "highpass", "dwt1_axis", "idwt1_axis", "dwt2", "idwt2",
    "level_shapes", "coeff_count", "sure_curve", "sure_threshold",
    "soft_threshold", "noise_estimate", "subspace", "hyres", "hyres_tiled",
    "tile_weights_1d", "oracle_gram", "hysime_rank", "truncation_df", "truncation_sure", "sure_rank",
]

# ---------------------------------------------------------------------------
# Wavelet filters (Daubechies' orthonormal family, 2 vanishing moments = 4 taps)
_S3 = math.sqrt(3.0)
DB2 = np.array([1.0 + _S3, 3.0 + _S3, 3.0 - _S3, 1.0 - _S3]) / (4.0 * math.sqrt(2.0))
HAAR = np.array([1.0, 1.0]) / math.sqrt(2.0)


def highpass(h: np.ndarray) -> np.ndarray:
    """Quadrature-mirror high-pass filter g[m] = (-1)^m h[K-1-m]."""
    K = len(h)
    return np.array([(-1.0) ** m * h[K - 1 - m] for m in range(K)])


def _ext_len(N: int) -> int:
    return N + (N & 1)


def dwt1_axis(x: np.ndarray, axis: int, h: np.ndarray = DB2) -> Tuple[np.ndarray, np.ndarray]:
    """One analysis step along ``axis`` with periodic extension.

    An odd-length axis is first extended by a copy of its last sample.  Then
    a[k] = sum_m h[m] x[(2k+m) mod N'], d[k] = sum_m g[m] x[(2k+m) mod N'].
    """
    x = np.moveaxis(np.asarray(x, dtype=np.float64), axis, 0)
    N = x.shape[0]
    if N & 1:
        x = np.concatenate([x, x[-1:]], axis=0)
    Ne = x.shape[0]
    g = highpass(h)
    half = Ne // 2
    k = np.arange(half)
    a = np.zeros((half,) + x.shape[1:])
    d = np.zeros((half,) + x.shape[1:])
    for m in range(len(h)):
        idx = (2 * k + m) % Ne
        a += h[m] * x[idx]
        d += g[m] * x[idx]
    return np.moveaxis(a, 0, axis), np.moveaxis(d, 0, axis)


def idwt1_axis(a: np.ndarray, d: np.ndarray, N: int, axis: int,
               h: np.ndarray = DB2) -> np.ndarray:
    """Synthesis step (transpose of the periodic analysis), cropped to N.

    x[(2k+m) mod N'] += h[m] a[k] + g[m] d[k] for every k and tap m.
    """
    a = np.moveaxis(np.asarray(a, dtype=np.float64), axis, 0)
    d = np.moveaxis(np.asarray(d, dtype=np.float64), axis, 0)
    Ne = _ext_len(N)
    assert a.shape[0] == Ne // 2
    g = highpass(h)
    x = np.zeros((Ne,) + a.shape[1:])
    k = np.arange(Ne // 2)
    for m in range(len(h)):
        idx = (2 * k + m) % Ne          # a permutation of one parity class
        x[idx] += h[m] * a + g[m] * d
    return np.moveaxis(x[:N], 0, axis)


def level_shapes(H: int, W: int, L: int) -> List[Tuple[int, int]]:
    """Sizes (h_l, w_l) of the approximation after each level l = 1..L."""
    out = []
    h, w = H, W
    for _ in range(L):
        h, w = (h + 1) // 2, (w + 1) // 2
        out.append((h, w))
    return out


def coeff_count(H: int, W: int, L: int) -> int:
    sh = level_shapes(H, W, L)
    return sum(3 * h * w for h, w in sh) + sh[-1][0] * sh[-1][1]


def dwt2(img: np.ndarray, L: int, h: np.ndarray = DB2) -> np.ndarray:
    """L-level 2-D transform of one image; returns the flat coefficient vector.

    Each level filters rows (along x) then columns (along y).  Layout:
    [LH_1, HL_1, HH_1, LH_2, HL_2, HH_2, ..., LL_L], each block row-major,
    where the first letter is the filter along y and the second along x.
    """
    cur = np.asarray(img, dtype=np.float64)
    parts = []
    for _ in range(L):
        lo_x, hi_x = dwt1_axis(cur, 1, h)
        ll, hl = dwt1_axis(lo_x, 0, h)
        lh, hh = dwt1_axis(hi_x, 0, h)
        parts += [lh.ravel(), hl.ravel(), hh.ravel()]
        cur = ll
    parts.append(cur.ravel())
    return np.concatenate(parts)


def idwt2(coeffs: np.ndarray, H: int, W: int, L: int, h: np.ndarray = DB2) -> np.ndarray:
    """Inverse of :func:`dwt2` (coarsest level first)."""
    sh = level_shapes(H, W, L)
    sizes = [(H, W)] + sh
    offs = []
    o = 0
    for (hl, wl) in sh:
        offs.append(o)
        o += 3 * hl * wl
    hL, wL = sh[-1]
    cur = coeffs[o:o + hL * wL].reshape(hL, wL).astype(np.float64)
    for lev in range(L - 1, -1, -1):
        hl, wl = sh[lev]
        Hp, Wp = sizes[lev]
        base = offs[lev]
        blk = hl * wl
        lh = coeffs[base:base + blk].reshape(hl, wl)
        hl_ = coeffs[base + blk:base + 2 * blk].reshape(hl, wl)
        hh = coeffs[base + 2 * blk:base + 3 * blk].reshape(hl, wl)
        lo_x = idwt1_axis(cur, hl_, Hp, 0, h)
        hi_x = idwt1_axis(lh, hh, Hp, 0, h)
        cur = idwt1_axis(lo_x, hi_x, Wp, 1, h)
    return cur


# ---------------------------------------------------------------------------
# Thresholding
def soft_threshold(b: np.ndarray, lam: float) -> np.ndarray:
    """sign(b) * max(|b| - lam, 0); zero at |b| == lam."""
    return np.sign(b) * np.maximum(np.abs(b) - lam, 0.0)


def sure_curve(b: np.ndarray) -> Tuple[np.ndarray, np.ndarray]:
    """SURE of soft thresholding at unit noise for every candidate threshold.

    With a_1 <= ... <= a_N the sorted magnitudes and a_0 = 0,
    S_j = N - 2 j + sum_{k<=j} a_k^2 + (N - j) a_j^2 is the risk estimate
    N - 2 #{|b| <= t} + sum min(b^2, t^2) evaluated at t = a_j.
    Returns (candidates a_0..a_N, S_0..S_N).
    """
    a = np.sort(np.abs(np.asarray(b, dtype=np.float64).ravel()))
    N = a.size
    a = np.concatenate([[0.0], a])
    j = np.arange(N + 1, dtype=np.float64)
    cs = np.cumsum(a * a)
    S = N - 2.0 * j + cs + (N - j) * a * a
    return a, S


def sure_threshold(b: np.ndarray) -> Tuple[float, float]:
    """(lambda, SURE(lambda)): first minimiser over the candidate set."""
    a, S = sure_curve(b)
    j = int(np.argmin(S))
    return float(a[j]), float(S[j])


def sure_at(b: np.ndarray, t: float) -> float:
    """SURE(t) = N - 2 #{|b| <= t} + sum min(b^2, t^2) (definition)."""
    ab = np.abs(np.asarray(b, dtype=np.float64).ravel())
    return float(ab.size - 2.0 * np.count_nonzero(ab <= t) + np.minimum(ab * ab, t * t).sum())


# ---------------------------------------------------------------------------
# Noise and subspace
def oracle_gram(Y2: np.ndarray) -> np.ndarray:
    Y2 = np.asarray(Y2, dtype=np.float64)
    return Y2.T @ Y2


def noise_estimate(Y2: np.ndarray, G: Optional[np.ndarray] = None) -> np.ndarray:
    """sigma_i = sqrt(RSS_i / n), RSS_i of band i regressed on the others.

    The least-squares coefficients solve the normal equations
    (Y_{-i}^T Y_{-i}) beta = Y_{-i}^T y_i; RSS = y_i^T y_i - y_i^T Y_{-i} beta.
    """
    Y2 = np.asarray(Y2, dtype=np.float64)
    n, p = Y2.shape
    if G is None:
        G = oracle_gram(Y2)
    sig = np.empty(p)
    for i in range(p):
        o = np.r_[0:i, i + 1:p]
        Goo = G[np.ix_(o, o)]
        goi = G[o, i]
        beta = np.linalg.solve(Goo, goi)
        rss = G[i, i] - goi @ beta
        if not rss > 0:
            raise FloatingPointError("band %d is an exact combination of the others" % i)
        sig[i] = math.sqrt(rss / n)
    return sig


def _sign_fix(V: np.ndarray) -> np.ndarray:
    V = V.copy()
    for i in range(V.shape[1]):
        k = int(np.argmax(np.abs(V[:, i])))
        if V[k, i] < 0:
            V[:, i] = -V[:, i]
    return V


def subspace(Yw: np.ndarray, r: int) -> Tuple[np.ndarray, np.ndarray]:
    """Top-r eigenvectors (sign-fixed) and all eigenvalues (descending) of Yw^T Yw."""
    C = Yw.T @ Yw
    w, U = np.linalg.eigh(C)
    order = np.argsort(w)[::-1]
    w = w[order]
    U = U[:, order]
    return _sign_fix(U[:, :r]), w


# ---------------------------------------------------------------------------
# Rank selection: the subspace dimension chosen from the data
def hysime_rank(evals: np.ndarray, n: int, r_max: int) -> int:
    """HySime subspace identification applied to the whitened cube.

    HySime keeps the eigen-directions e of the signal correlation (data
    correlation R_y minus noise correlation R_n) along which the data power
    e^T R_y e exceeds twice the noise power e^T R_n e: including e changes the
    mean-square error of the projection estimate by -e^T R_y e + 2 e^T R_n e.
    After whitening by the per-band noise levels, R_n = I and R_y = C / n, so
    the directions are the eigenvectors of C and the change is 2 - lambda / n.
    The count is capped to [1, r_max].
    """
    delta = 2.0 - np.asarray(evals, dtype=np.float64) / float(n)
    k = int(np.sum(delta < 0.0))
    return min(max(k, 1), int(r_max))


def truncation_df(evals: np.ndarray, n: int, r: int) -> float:
    """Divergence (degrees of freedom) of the rank-r truncated SVD of an
    n x p matrix (n >= p, distinct singular values), in terms of the squared
    singular values lambda (the eigenvalues of its Gram, descending):
        r (n - p + 1) + r (r - 1) + 2 sum_{i <= r < j} lambda_i / (lambda_i - lambda_j),
    the spectral-estimator divergence sum_i [f_i' + (n - p) f_i / s_i] +
    2 sum_{i != j} s_i f_i / (s_i^2 - s_j^2) with f_i = s_i for i <= r, else 0."""
    lam = np.asarray(evals, dtype=np.float64)
    p = lam.size
    df = r * (n - p + 1) + r * (r - 1)
    for i in range(r):
        for j in range(r, p):
            df += 2.0 * lam[i] / (lam[i] - lam[j])
    return float(df)


def truncation_sure(evals: np.ndarray, n: int, r: int) -> float:
    """Stein's unbiased risk estimate (unit noise) of the rank-r truncation of
    the whitened n x p cube: ||Yw - Yw_r||^2 - n p + 2 df(r), where the
    residual is the sum of the discarded eigenvalues."""
    lam = np.asarray(evals, dtype=np.float64)
    p = lam.size
    return float(np.sum(lam[r:]) - n * p + 2.0 * truncation_df(lam, n, r))


def sure_rank(evals: np.ndarray, n: int, r_max: int) -> int:
    """The rank in [1, r_max] minimising truncation_sure (smallest on ties)."""
    vals = [truncation_sure(evals, n, r) for r in range(1, int(r_max) + 1)]
    return 1 + int(np.argmin(vals))


# ---------------------------------------------------------------------------
# The whole denoiser
def hyres(Y: np.ndarray, r: int, L: int, sigma: Optional[np.ndarray] = None,
          lam: Optional[Sequence[float]] = None, V: Optional[np.ndarray] = None,
          h: np.ndarray = DB2, detail_only: bool = False,
          rank_rule: Optional[str] = None) -> Dict[str, np.ndarray]:
    """Run O1..O10 on an H x W x p cube.  Everything is float64.

    ``sigma``, ``lam`` and ``V`` may be supplied to bypass their estimation.
    ``rank_rule`` "hysime" or "sure": ``r`` is the largest rank, and the rank
    used is chosen from the eigenvalues of the whitened Gram (hysime_rank,
    sure_rank); the result then carries ``rank``.
    Returns a dict with X (denoised, H x W x p), sigma, V, evals (all,
    descending, of the whitened Gram), lam, sure (minimum SURE per component),
    gap (evals[r-1] / evals[r]), Z (component images), B (coefficients).
    """
    Y = np.asarray(Y, dtype=np.float64)
    H, W, p = Y.shape
    n = H * W
    Y2 = Y.reshape(n, p)                                         # O1
    if sigma is None:
        sigma = noise_estimate(Y2)                               # O2
    sigma = np.asarray(sigma, dtype=np.float64)
    Yw = Y2 / sigma[None, :]                                     # O3
    rank = None
    if rank_rule is not None:
        if V is not None:
            raise ValueError("a given basis fixes the rank")
        _, ev_all = subspace(Yw, 1)
        rank = hysime_rank(ev_all, n, r) if rank_rule == "hysime" else sure_rank(ev_all, n, r)
        r = rank
    if V is None:
        V, evals = subspace(Yw, r)                               # O4
    else:
        evals = np.linalg.eigvalsh(Yw.T @ Yw)[::-1]
    Z = Yw @ V                                                   # O5
    Nc = coeff_count(H, W, L)
    hL, wL = level_shapes(H, W, L)[-1]
    B = np.empty((r, Nc))
    Zh = np.empty((r, H, W))
    lam_out = np.empty(r)
    sure_out = np.empty(r)
    for i in range(r):
        b = dwt2(Z[:, i].reshape(H, W), L, h)                    # O6
        B[i] = b
        sel = b[: Nc - hL * wL] if detail_only else b
        if lam is None:
            li, si = sure_threshold(sel)                         # O7
        else:
            li = float(lam[i])
            si = sure_at(sel, li)
        lam_out[i] = li
        sure_out[i] = si
        bt = soft_threshold(b, li)                               # O8
        if detail_only:
            bt[Nc - hL * wL:] = b[Nc - hL * wL:]
        Zh[i] = idwt2(bt, H, W, L, h)                            # O9
    Xw = Zh.reshape(r, n).T @ V.T                                # O10
    X = (Xw * sigma[None, :]).reshape(H, W, p)
    gap = evals[r - 1] / evals[r] if r < p else float("inf")
    out = dict(X=X, sigma=sigma, V=V, evals=evals, lam=lam_out, sure=sure_out,
               gap=gap, Z=Z.T.reshape(r, H, W), B=B)
    if rank is not None:
        out["rank"] = rank
    return out


# ---------------------------------------------------------------------------
# Sliding-window form
def tile_weights_1d(start: int, tile: int, size: int, overlap: int) -> np.ndarray:
    """Blend weight of one tile along one axis (length ``tile``).

    It ramps up over the tile's first ``overlap`` samples and down over its
    last ``overlap`` samples as sin^2(pi/2 (k + 1/2) / overlap); there is no
    ramp on a side that touches the image border.
    """
    w = np.ones(tile)
    k = np.arange(overlap)
    ramp = np.sin(0.5 * np.pi * (k + 0.5) / overlap) ** 2
    if start > 0:
        w[:overlap] = ramp
    if start + tile < size:
        w[tile - overlap:] = ramp[::-1]
    return w


def hyres_tiled(Y: np.ndarray, r: int, L: int, tile: int, overlap: int,
                starts_y: Sequence[int], starts_x: Sequence[int],
                tile_fn=None) -> np.ndarray:
    """Denoise every tile independently and blend: sum_t w_t X_t / sum_t w_t.

    ``tile_fn(Y_tile) -> X_tile`` replaces the per-tile denoiser (for tests).
    """
    Y = np.asarray(Y, dtype=np.float64)
    H, W, p = Y.shape
    th, tw = min(tile, H), min(tile, W)
    acc = np.zeros((H, W, p))
    wsum = np.zeros((H, W))
    for sy in starts_y:
        wy = tile_weights_1d(sy, th, H, overlap)
        for sx in starts_x:
            wx = tile_weights_1d(sx, tw, W, overlap)
            sub = Y[sy:sy + th, sx:sx + tw]
            out = hyres(sub, r, L)["X"] if tile_fn is None else tile_fn(sub)
            w2 = wy[:, None] * wx[None, :]
            acc[sy:sy + th, sx:sx + tw] += w2[:, :, None] * out
            wsum[sy:sy + th, sx:sx + tw] += w2
    return acc / wsum[:, :, None]
