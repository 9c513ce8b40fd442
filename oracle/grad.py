"""Differentiable FP64 CPU oracle of HyRes (test infrastructure only).

The same steps as :mod:`oracle.hyres_oracle` (O1..O10), re-expressed with
plain PyTorch CPU float64 operations so that torch's autograd supplies a
gradient that is independent of the hand-written adjoint of the HIP path.
The thresholds are inputs (a stop-gradient through the SURE argmin): the
gradient is taken with respect to the cube and to the thresholds.

Only the test suite imports this module.
"""
from __future__ import annotations

import math
from typing import Tuple

import torch

from .hyres_oracle import DB2, highpass, level_shapes


def _filters(dtype=torch.float64):
    h = torch.tensor(DB2, dtype=dtype)
    g = torch.tensor(highpass(DB2), dtype=dtype)
    return h, g


def dwt1(x: torch.Tensor, axis: int) -> Tuple[torch.Tensor, torch.Tensor]:
    h, g = _filters(x.dtype)
    x = x.movedim(axis, 0)
    N = x.shape[0]
    if N % 2:
        x = torch.cat([x, x[-1:]], 0)
    Ne = x.shape[0]
    k = torch.arange(Ne // 2)
    a = 0
    d = 0
    for m in range(4):
        xi = x[(2 * k + m) % Ne]
        a = a + h[m] * xi
        d = d + g[m] * xi
    return a.movedim(0, axis), d.movedim(0, axis)


def idwt1(a: torch.Tensor, d: torch.Tensor, N: int, axis: int) -> torch.Tensor:
    h, g = _filters(a.dtype)
    a = a.movedim(axis, 0)
    d = d.movedim(axis, 0)
    Ne = N + (N % 2)
    k = torch.arange(Ne // 2)
    x = torch.zeros((Ne,) + tuple(a.shape[1:]), dtype=a.dtype)
    for m in range(4):
        idx = (2 * k + m) % Ne
        x = x.index_add(0, idx, h[m] * a + g[m] * d)
    return x[:N].movedim(0, axis)


def dwt2(img: torch.Tensor, L: int):
    cur = img
    parts = []
    for _ in range(L):
        lo_x, hi_x = dwt1(cur, 1)
        ll, hl = dwt1(lo_x, 0)
        lh, hh = dwt1(hi_x, 0)
        parts.append((lh, hl, hh))
        cur = ll
    return parts, cur


def idwt2(parts, ll, H: int, W: int, L: int):
    sizes = [(H, W)] + level_shapes(H, W, L)
    cur = ll
    for lev in range(L - 1, -1, -1):
        lh, hl, hh = parts[lev]
        Hp, Wp = sizes[lev]
        lo_x = idwt1(cur, hl, Hp, 0)
        hi_x = idwt1(lh, hh, Hp, 0)
        cur = idwt1(lo_x, hi_x, Wp, 1)
    return cur


def soft(b: torch.Tensor, lam: torch.Tensor) -> torch.Tensor:
    return torch.sign(b) * torch.relu(b.abs() - lam)


def noise_sigma(Y2: torch.Tensor) -> torch.Tensor:
    """sigma_i = sqrt(RSS_i / n) from the per-band normal equations."""
    n, p = Y2.shape
    G = Y2.T @ Y2
    out = []
    for i in range(p):
        o = [j for j in range(p) if j != i]
        Goo = G[o][:, o]
        goi = G[o, i]
        beta = torch.linalg.solve(Goo, goi)
        out.append(torch.sqrt((G[i, i] - goi @ beta) / n))
    return torch.stack(out)


def hyres_forward(Y: torch.Tensor, lam: torch.Tensor, r: int, L: int,
                  sign_ref: torch.Tensor = None) -> torch.Tensor:
    """Denoised cube for thresholds ``lam`` (float64 CPU tensors).

    ``sign_ref`` (p x r) fixes the eigenvector signs to agree with a reference
    basis, so that finite differences see a smooth function.
    """
    H, W, p = Y.shape
    n = H * W
    Y2 = Y.reshape(n, p)
    sig = noise_sigma(Y2)
    Yw = Y2 / sig
    C = Yw.T @ Yw
    w, U = torch.linalg.eigh(C)
    V = U.flip(1)[:, :r]
    if sign_ref is None:
        idx = V.abs().argmax(0)
        s = torch.sign(V[idx, torch.arange(r)]).detach()
    else:
        s = torch.sign((V * sign_ref).sum(0)).detach()
    V = V * s
    Z = (Yw @ V).T.reshape(r, H, W)
    outs = []
    for i in range(r):
        parts, ll = dwt2(Z[i], L)
        parts = [tuple(soft(t, lam[i]) for t in blk) for blk in parts]
        ll = soft(ll, lam[i])
        outs.append(idwt2(parts, ll, H, W, L))
    Zh = torch.stack(outs).reshape(r, n)
    X = (Zh.T @ V.T) * sig
    return X.reshape(H, W, p)
