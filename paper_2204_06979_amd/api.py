"""Python binding of libhyres (torch tensors in, torch tensors out).

PyTorch provides device memory and the current stream; every computation
runs in the library's HIP kernels.  All calls are asynchronous on
``torch.cuda.current_stream()``; the returned ``info`` tensors are filled
when that stream reaches them.
"""
from __future__ import annotations

import ctypes as C
from typing import Dict, Optional, Tuple

import torch

from . import _lib as L

_HANDLES: Dict[int, int] = {}


def _handle(device: torch.device) -> int:
    idx = device.index if device.index is not None else torch.cuda.current_device()
    h = _HANDLES.get(idx)
    if h is None:
        hp = C.c_void_p()
        L.check(L.lib().hyres_create(C.byref(hp), idx), "hyres_create")
        h = hp.value
        _HANDLES[idx] = h
    return h


def _stream(device: torch.device) -> int:
    return torch.cuda.current_stream(device).cuda_stream


def _dtype_code(t: torch.Tensor) -> int:
    if t.dtype == torch.float32:
        return L.HYRES_F32
    if t.dtype == torch.float64:
        return L.HYRES_F64
    raise TypeError("cubes must be float32 or float64, got %s" % t.dtype)


def _workspace(nbytes: int, device: torch.device) -> Tuple[torch.Tensor, int]:
    buf = torch.empty(int(nbytes) + 256, dtype=torch.uint8, device=device)
    ptr = buf.data_ptr()
    off = (-ptr) % 256
    return buf, ptr + off


def _cube_strides(Y: torch.Tensor) -> Tuple[int, int]:
    if Y.dim() != 3:
        raise ValueError("cube must be H x W x p")
    if Y.stride(2) != 1:
        raise ValueError("the band axis must be contiguous (band-fastest layout)")
    return Y.stride(1), Y.stride(0)


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else t.data_ptr()


def _need_cuda(t: torch.Tensor, name: str) -> None:
    if not t.is_cuda:
        raise ValueError("%s must be a GPU tensor" % name)


def _flags(all_evals: bool, rank_rule: Optional[str]) -> int:
    f = L.FLAG_ALL_EVALS if all_evals else 0
    if rank_rule == "hysime":
        f |= L.FLAG_RANK_HYSIME
    elif rank_rule == "sure":
        f |= L.FLAG_RANK_SURE
    elif rank_rule is not None:
        raise ValueError("rank_rule must be None, 'hysime' or 'sure'")
    return f


def coeff_count(H: int, W: int, levels: int) -> int:
    n = L.lib().hyres_coeff_count(H, W, levels)
    if n <= 0:
        raise ValueError("invalid transform shape %dx%d, %d levels" % (H, W, levels))
    return int(n)


def estimate_noise(Y: torch.Tensor, return_gram: bool = False):
    """Per-band noise std by regression on the other bands (device FP64)."""
    _need_cuda(Y, "Y")
    H, W, p = Y.shape
    pitch, rp = _cube_strides(Y)
    dt = _dtype_code(Y)
    lib = L.lib()
    nb = C.c_size_t()
    L.check(lib.hyres_estimate_noise_workspace_size(H, W, p, dt, C.byref(nb)), "workspace size")
    buf, ws = _workspace(nb.value, Y.device)
    sigma = torch.empty(p, dtype=torch.float64, device=Y.device)
    gram = torch.empty(p, p, dtype=torch.float64, device=Y.device) if return_gram else None
    status = torch.zeros(1, dtype=torch.int32, device=Y.device)
    L.check(lib.hyres_estimate_noise(_handle(Y.device), Y.data_ptr(), H, W, p, pitch, rp, dt,
                                     sigma.data_ptr(), _ptr(gram), status.data_ptr(), ws, nb.value,
                                     _stream(Y.device)), "hyres_estimate_noise")
    return (sigma, gram, status) if return_gram else (sigma, status)


def subspace(Y: torch.Tensor, rank: int, sigma: Optional[torch.Tensor] = None):
    """Top-r eigenvectors (p x r) and all eigenvalues of the whitened Gram."""
    _need_cuda(Y, "Y")
    H, W, p = Y.shape
    pitch, rp = _cube_strides(Y)
    dt = _dtype_code(Y)
    lib = L.lib()
    nb = C.c_size_t()
    L.check(lib.hyres_subspace_workspace_size(H, W, p, rank, dt, C.byref(nb)), "workspace size")
    buf, ws = _workspace(nb.value, Y.device)
    Vt = torch.empty(rank, p, dtype=torch.float64, device=Y.device)     # column-major p x r
    ev = torch.empty(p, dtype=torch.float64, device=Y.device)
    status = torch.zeros(1, dtype=torch.int32, device=Y.device)
    sg = None if sigma is None else sigma.to(device=Y.device, dtype=torch.float64).contiguous()
    L.check(lib.hyres_subspace(_handle(Y.device), Y.data_ptr(), H, W, p, pitch, rp, dt, _ptr(sg), rank,
                               Vt.data_ptr(), ev.data_ptr(), status.data_ptr(), ws, nb.value,
                               _stream(Y.device)), "hyres_subspace")
    return Vt.T, ev, status


def dwt2(x: torch.Tensor, levels: int) -> torch.Tensor:
    """Batched L-level periodised db2 transform: (B, H, W) -> (B, Nc)."""
    _need_cuda(x, "x")
    x = x.contiguous()
    B, H, W = x.shape
    dt = _dtype_code(x)
    lib = L.lib()
    nb = C.c_size_t()
    L.check(lib.hyres_dwt2_workspace_size(B, H, W, levels, dt, C.byref(nb)), "workspace size")
    buf, ws = _workspace(nb.value, x.device)
    out = torch.empty(B, coeff_count(H, W, levels), dtype=x.dtype, device=x.device)
    L.check(lib.hyres_dwt2(_handle(x.device), x.data_ptr(), B, H, W, levels, dt, out.data_ptr(), ws,
                           nb.value, _stream(x.device)), "hyres_dwt2")
    return out


def idwt2(coeffs: torch.Tensor, H: int, W: int, levels: int, lam: Optional[torch.Tensor] = None,
          scope: str = "all") -> torch.Tensor:
    """Inverse transform (optionally soft-thresholding with per-image lambda)."""
    _need_cuda(coeffs, "coeffs")
    coeffs = coeffs.contiguous()
    B = coeffs.shape[0]
    dt = _dtype_code(coeffs)
    lib = L.lib()
    nb = C.c_size_t()
    L.check(lib.hyres_dwt2_workspace_size(B, H, W, levels, dt, C.byref(nb)), "workspace size")
    buf, ws = _workspace(nb.value, coeffs.device)
    out = torch.empty(B, H, W, dtype=coeffs.dtype, device=coeffs.device)
    lm = None if lam is None else lam.to(device=coeffs.device, dtype=torch.float64).contiguous()
    sc = L.SCOPE_ALL if scope == "all" else L.SCOPE_DETAIL
    L.check(lib.hyres_idwt2(_handle(coeffs.device), coeffs.data_ptr(), B, H, W, levels, dt, _ptr(lm), sc,
                            out.data_ptr(), ws, nb.value, _stream(coeffs.device)), "hyres_idwt2")
    return out


def sure_threshold(coeffs: torch.Tensor):
    """Exact SURE-minimising soft threshold of each row of a (B, N) tensor."""
    _need_cuda(coeffs, "coeffs")
    if coeffs.stride(1) != 1:
        coeffs = coeffs.contiguous()
    B, N = coeffs.shape
    dt = _dtype_code(coeffs)
    lib = L.lib()
    nb = C.c_size_t()
    L.check(lib.hyres_sure_workspace_size(B, N, dt, C.byref(nb)), "workspace size")
    buf, ws = _workspace(nb.value, coeffs.device)
    lam = torch.empty(B, dtype=torch.float64, device=coeffs.device)
    sure = torch.empty(B, dtype=torch.float64, device=coeffs.device)
    status = torch.zeros(1, dtype=torch.int32, device=coeffs.device)
    row_stride = coeffs.stride(0) if B > 1 else N         # torch may report any stride for a size-1 dim
    L.check(lib.hyres_sure_threshold(_handle(coeffs.device), coeffs.data_ptr(), B, N, row_stride, dt,
                                     lam.data_ptr(), sure.data_ptr(), status.data_ptr(), ws, nb.value,
                                     _stream(coeffs.device)), "hyres_sure_threshold")
    return lam, sure, status


class Denoiser:
    """A reusable single-cube solve: workspace and output buffers are allocated
    once, so ``run`` only enqueues kernels (and can be captured in a graph)."""

    def __init__(self, H: int, W: int, p: int, rank: int, levels: int, dtype=torch.float32,
                 precision: str = "native", scope: str = "all", device=None, all_evals: bool = False,
                 rank_rule: Optional[str] = None, check_eigs: bool = False):
        self.device = torch.device(device if device is not None else "cuda")
        self.H, self.W, self.p, self.r, self.L = H, W, p, rank, levels
        self.dtype = dtype
        self.dt = L.HYRES_F32 if dtype == torch.float32 else L.HYRES_F64
        self.opt = L.Options(rank, levels, L.PREC_MIXED if precision == "mixed" else L.PREC_NATIVE,
                             L.SCOPE_ALL if scope == "all" else L.SCOPE_DETAIL, _flags(all_evals, rank_rule))
        lib = L.lib()
        nb = C.c_size_t()
        L.check(lib.hyres_denoise_workspace_size(H, W, p, C.byref(self.opt), self.dt, C.byref(nb)),
                "workspace size")
        self.ws_bytes = nb.value
        self._buf, self._ws = _workspace(nb.value, self.device)
        dev = self.device
        self.sigma = torch.empty(p, dtype=torch.float64, device=dev)
        self.V = torch.empty(rank, p, dtype=torch.float64, device=dev)
        self.evals = torch.empty(p, dtype=torch.float64, device=dev)
        self.lam = torch.empty(rank, dtype=torch.float64, device=dev)
        self.sure = torch.empty(rank, dtype=torch.float64, device=dev)
        self.gap = torch.empty(1, dtype=torch.float64, device=dev)
        self.status = torch.zeros(1, dtype=torch.int32, device=dev)
        self.rank = torch.zeros(1, dtype=torch.int32, device=dev)
        self.eig_check = torch.zeros(2, dtype=torch.float64, device=dev) if check_eigs else None
        self.out = L.Outputs(self.sigma.data_ptr(), self.V.data_ptr(), self.evals.data_ptr(),
                             self.lam.data_ptr(), self.sure.data_ptr(), self.gap.data_ptr(),
                             self.status.data_ptr(), self.rank.data_ptr(), _ptr(self.eig_check))
        self.X = torch.empty(H, W, p, dtype=dtype, device=dev)

    def run(self, Y: torch.Tensor, sigma: Optional[torch.Tensor] = None,
            lam: Optional[torch.Tensor] = None, X: Optional[torch.Tensor] = None) -> torch.Tensor:
        pitch, rp = _cube_strides(Y)
        X = self.X if X is None else X
        xp, xrp = _cube_strides(X)
        L.check(L.lib().hyres_denoise(_handle(self.device), Y.data_ptr(), self.H, self.W, self.p, pitch, rp,
                                      self.dt, C.byref(self.opt), _ptr(sigma), _ptr(lam), X.data_ptr(), xp,
                                      xrp, C.byref(self.out), self._ws, self.ws_bytes,
                                      _stream(self.device)), "hyres_denoise")
        return X

    def run_hyminor(self, Y: torch.Tensor, l1: "L.L1Options", sigma: Optional[torch.Tensor] = None,
                    lam: Optional[torch.Tensor] = None, X: Optional[torch.Tensor] = None) -> torch.Tensor:
        """HyRes, then the sparse-noise stage in place in X (hyres_hyminor)."""
        pitch, rp = _cube_strides(Y)
        X = self.X if X is None else X
        xp, xrp = _cube_strides(X)
        L.check(L.lib().hyres_hyminor(_handle(self.device), Y.data_ptr(), self.H, self.W, self.p, pitch, rp,
                                      self.dt, C.byref(self.opt), _ptr(sigma), _ptr(lam), C.byref(l1),
                                      X.data_ptr(), xp, xrp, C.byref(self.out), self._ws, self.ws_bytes,
                                      _stream(self.device)), "hyres_hyminor")
        return X

    def info(self) -> Dict[str, torch.Tensor]:
        info = dict(sigma=self.sigma, V=self.V.T, evals=self.evals, lam=self.lam, sure=self.sure,
                    gap=self.gap, status=self.status, rank=self.rank)
        if self.eig_check is not None:
            info["eig_resid"], info["eig_orth"] = self.eig_check[0:1], self.eig_check[1:2]
        return info


def denoise(Y: torch.Tensor, rank: int, levels: int, precision: str = "native",
            sigma: Optional[torch.Tensor] = None, lam: Optional[torch.Tensor] = None,
            scope: str = "all", all_evals: bool = False, rank_rule: Optional[str] = None,
            check_eigs: bool = False):
    """HyRes denoising of one H x W x p cube; returns (X, info).  With
    ``rank_rule`` ("hysime" or "sure") ``rank`` is the largest rank and
    info["rank"] the one the device chose.  With ``check_eigs`` info also holds
    the eigensolve's relative residual ``eig_resid`` and orthonormality error
    ``eig_orth``."""
    _need_cuda(Y, "Y")
    H, W, p = Y.shape
    dn = Denoiser(H, W, p, rank, levels, dtype=Y.dtype, precision=precision, scope=scope, device=Y.device,
                  all_evals=all_evals, rank_rule=rank_rule, check_eigs=check_eigs)
    sg = None if sigma is None else sigma.to(device=Y.device, dtype=torch.float64).contiguous()
    lm = None if lam is None else lam.to(device=Y.device, dtype=torch.float64).contiguous()
    X = dn.run(Y, sg, lm)
    return X, dn.info()


def l1l1_spectral(Hc: torch.Tensor, lam: float = 1.0, mu1: float = 1.0, mu2: float = 1.0, iters: int = 50,
                  X: Optional[torch.Tensor] = None) -> torch.Tensor:
    """HyMiNoR's sparse-noise stage alone: per pixel spectrum h of the
    H x W x p cube ``Hc``, ``iters`` split-Bregman sweeps of
    argmin_x ||h - x||_1 + lam ||D x||_1 (D the first-order spectral
    difference; penalties mu1, mu2).  ``X`` may be ``Hc`` (in place)."""
    _need_cuda(Hc, "Hc")
    H, W, p = Hc.shape
    X = torch.empty_like(Hc) if X is None else X
    pitch, rp = _cube_strides(Hc)
    xp, xrp = _cube_strides(X)
    o = L.L1Options(float(lam), float(mu1), float(mu2), int(iters))
    L.check(L.lib().hyres_l1l1_spectral(_handle(Hc.device), Hc.data_ptr(), H, W, p, pitch, rp, _dtype_code(Hc),
                                        C.byref(o), X.data_ptr(), xp, xrp, _stream(Hc.device)),
            "hyres_l1l1_spectral")
    return X


def hyminor(Y: torch.Tensor, rank: int, levels: int, lam: float = 1.0, mu1: float = 1.0, mu2: float = 1.0,
            iters: int = 50, precision: str = "native", sigma: Optional[torch.Tensor] = None,
            hyres_lam: Optional[torch.Tensor] = None, rank_rule: Optional[str] = None):
    """HyMiNoR: HyRes of the cube, then the sparse-noise stage on its output;
    returns (X, info) with info describing the HyRes stage."""
    _need_cuda(Y, "Y")
    H, W, p = Y.shape
    dn = Denoiser(H, W, p, rank, levels, dtype=Y.dtype, precision=precision, device=Y.device,
                  rank_rule=rank_rule)
    sg = None if sigma is None else sigma.to(device=Y.device, dtype=torch.float64).contiguous()
    lm = None if hyres_lam is None else hyres_lam.to(device=Y.device, dtype=torch.float64).contiguous()
    X = dn.run_hyminor(Y, L.L1Options(float(lam), float(mu1), float(mu2), int(iters)), sg, lm)
    return X, dn.info()


def wsrrr(Y: torch.Tensor, rank: int, levels: int, iters: int = 5, sigma: Optional[torch.Tensor] = None,
          lam: Optional[torch.Tensor] = None, scope: str = "all"):
    """WSRRR of one H x W x p cube (hyres_wsrrr): HyRes, then ``iters``
    alternations of the Procrustes step for the subspace and the
    soft-threshold step for the wavelet coefficients at HyRes's thresholds.
    Returns (X, info) as ``denoise`` (V: the final subspace)."""
    _need_cuda(Y, "Y")
    H, W, p = Y.shape
    dev = Y.device
    dt = _dtype_code(Y)
    lib = L.lib()
    opt = L.Options(rank, levels, L.PREC_NATIVE, L.SCOPE_ALL if scope == "all" else L.SCOPE_DETAIL, 0)
    nb = C.c_size_t()
    L.check(lib.hyres_wsrrr_workspace_size(H, W, p, C.byref(opt), dt, C.byref(nb)), "wsrrr workspace size")
    buf, ws = _workspace(nb.value, dev)
    o = dict(sigma=torch.empty(p, dtype=torch.float64, device=dev),
             V=torch.empty(rank, p, dtype=torch.float64, device=dev),
             evals=torch.empty(p, dtype=torch.float64, device=dev),
             lam=torch.empty(rank, dtype=torch.float64, device=dev),
             sure=torch.empty(rank, dtype=torch.float64, device=dev),
             gap=torch.empty(1, dtype=torch.float64, device=dev),
             status=torch.zeros(1, dtype=torch.int32, device=dev),
             rank=torch.zeros(1, dtype=torch.int32, device=dev))
    outs = L.Outputs(o["sigma"].data_ptr(), o["V"].data_ptr(), o["evals"].data_ptr(), o["lam"].data_ptr(),
                     o["sure"].data_ptr(), o["gap"].data_ptr(), o["status"].data_ptr(), o["rank"].data_ptr())
    X = torch.empty(H, W, p, dtype=Y.dtype, device=dev)
    sg = None if sigma is None else sigma.to(device=dev, dtype=torch.float64).contiguous()
    lm = None if lam is None else lam.to(device=dev, dtype=torch.float64).contiguous()
    pitch, rp = _cube_strides(Y)
    xp, xrp = _cube_strides(X)
    L.check(lib.hyres_wsrrr(_handle(dev), Y.data_ptr(), H, W, p, pitch, rp, dt, C.byref(opt), int(iters), _ptr(sg),
                            _ptr(lm), X.data_ptr(), xp, xrp, C.byref(outs), ws, nb.value, _stream(dev)),
            "hyres_wsrrr")
    del buf     # stream-ordered reuse by the caching allocator
    o["V"] = o["V"].T
    return X, o


def forpdn(Y: torch.Tensor, levels: int, sigma: Optional[torch.Tensor] = None,
           lam: Optional[torch.Tensor] = None, X: Optional[torch.Tensor] = None):
    """FORPDN of one H x W x p cube (hyres_forpdn): whitened bands, the db2
    wavelet, and per wavelet group the first-order spectral roughness smoother
    with its threshold chosen by SURE.  Returns (X, info) with sigma, lam and
    sure (levels + 1 groups) and status."""
    _need_cuda(Y, "Y")
    H, W, p = Y.shape
    dev = Y.device
    dt = _dtype_code(Y)
    lib = L.lib()
    sg = None if sigma is None else sigma.to(device=dev, dtype=torch.float64).contiguous()
    lm = None if lam is None else lam.to(device=dev, dtype=torch.float64).contiguous()
    nb = C.c_size_t()
    L.check(lib.hyres_forpdn_workspace_size(H, W, p, levels, dt, int(sg is not None), C.byref(nb)),
            "forpdn workspace size")
    buf, ws = _workspace(nb.value, dev)
    X = torch.empty(H, W, p, dtype=Y.dtype, device=dev) if X is None else X
    info = dict(sigma=torch.empty(p, dtype=torch.float64, device=dev),
                lam=torch.empty(levels + 1, dtype=torch.float64, device=dev),
                sure=torch.empty(levels + 1, dtype=torch.float64, device=dev),
                status=torch.zeros(1, dtype=torch.int32, device=dev))
    pitch, rp = _cube_strides(Y)
    xp, xrp = _cube_strides(X)
    L.check(lib.hyres_forpdn(_handle(dev), Y.data_ptr(), H, W, p, pitch, rp, dt, levels, _ptr(sg), _ptr(lm),
                             X.data_ptr(), xp, xrp, info["sigma"].data_ptr(), info["lam"].data_ptr(),
                             info["sure"].data_ptr(), info["status"].data_ptr(), ws, nb.value, _stream(dev)),
            "hyres_forpdn")
    del buf     # stream-ordered reuse by the caching allocator
    return X, info


def denoise_noalloc(Y: torch.Tensor, rank: int, levels: int, precision: str = "native",
                    sigma: Optional[torch.Tensor] = None, lam: Optional[torch.Tensor] = None,
                    scope: str = "all", out: Optional[Dict[str, torch.Tensor]] = None,
                    X: Optional[torch.Tensor] = None):
    """``denoise`` through ``hyres_denoise_noalloc``: the library takes its scratch
    from a fixed per-device array instead of a workspace.  The caller may pass
    the output cube ``X`` and the ``out`` tensors (sigma, V (rank x p), evals,
    lam, sure, gap, status) so that the call itself allocates nothing; those it
    omits are allocated here, before the call."""
    _need_cuda(Y, "Y")
    H, W, p = Y.shape
    dev = Y.device
    dt = _dtype_code(Y)
    opt = L.Options(rank, levels, L.PREC_MIXED if precision == "mixed" else L.PREC_NATIVE,
                    L.SCOPE_ALL if scope == "all" else L.SCOPE_DETAIL, 0)
    o = dict(out) if out is not None else {}
    shapes = dict(sigma=(p,), V=(rank, p), evals=(p,), lam=(rank,), sure=(rank,), gap=(1,))
    for k, shp in shapes.items():
        if k not in o:
            o[k] = torch.empty(shp, dtype=torch.float64, device=dev)
    if "status" not in o:
        o["status"] = torch.zeros(1, dtype=torch.int32, device=dev)
    if X is None:
        X = torch.empty(H, W, p, dtype=Y.dtype, device=dev)
    sg = None if sigma is None else sigma.to(device=dev, dtype=torch.float64).contiguous()
    lm = None if lam is None else lam.to(device=dev, dtype=torch.float64).contiguous()
    pitch, rp = _cube_strides(Y)
    xp, xrp = _cube_strides(X)
    if "rank" not in o:
        o["rank"] = torch.zeros(1, dtype=torch.int32, device=dev)
    outs = L.Outputs(o["sigma"].data_ptr(), o["V"].data_ptr(), o["evals"].data_ptr(), o["lam"].data_ptr(),
                     o["sure"].data_ptr(), o["gap"].data_ptr(), o["status"].data_ptr(), o["rank"].data_ptr())
    L.check(L.lib().hyres_denoise_noalloc(_handle(dev), Y.data_ptr(), H, W, p, pitch, rp, dt, C.byref(opt),
                                          _ptr(sg), _ptr(lm), X.data_ptr(), xp, xrp, C.byref(outs),
                                          _stream(dev)), "hyres_denoise_noalloc")
    info = dict(o)
    info["V"] = o["V"].T
    return X, info


class Batch:
    """A planned batch of independent cubes (uneven H, W, p, rank, levels).

    The library builds the descriptor and work tables once (``hyres_batch_create``);
    ``run`` enqueues one solve of every cube as persistent launches,
    ``launch_graph`` replays the same sequence as one HIP graph, and
    ``autotune`` picks the transform tile shapes for this batch's level widths.
    Outputs live in ``self.X[i]`` and ``self.info(i)``.
    """

    def __init__(self, cubes, ranks, levels, precision: str = "native", scope: str = "all",
                 sigmas=None, lams=None, all_evals: bool = False, rank_rule: Optional[str] = None):
        if len(cubes) == 0:
            raise ValueError("empty batch")
        Y0 = cubes[0]
        _need_cuda(Y0, "cube 0")
        self.device = Y0.device
        self.dtype = Y0.dtype
        self.dt = _dtype_code(Y0)
        count = len(cubes)
        ranks = [int(ranks)] * count if isinstance(ranks, int) else [int(r) for r in ranks]
        levels = [int(levels)] * count if isinstance(levels, int) else [int(l) for l in levels]
        if len(ranks) != count or len(levels) != count:
            raise ValueError("ranks and levels need one entry per cube")
        self.opt = L.Options(0, 0, L.PREC_MIXED if precision == "mixed" else L.PREC_NATIVE,
                             L.SCOPE_ALL if scope == "all" else L.SCOPE_DETAIL, _flags(all_evals, rank_rule))
        dev = self.device
        self.Y = list(cubes)
        self.X, self._info, self._keep = [], [], []
        arr = (L.Cube * count)()
        for i, Y in enumerate(cubes):
            _need_cuda(Y, "cube %d" % i)
            if Y.dtype != self.dtype or Y.device != dev:
                raise ValueError("every cube of a batch has the same dtype and device")
            H, W, p = Y.shape
            pitch, rp = _cube_strides(Y)
            r = ranks[i]
            X = torch.empty(H, W, p, dtype=self.dtype, device=dev)
            inf = dict(sigma=torch.empty(p, dtype=torch.float64, device=dev),
                       V=torch.empty(r, p, dtype=torch.float64, device=dev),
                       evals=torch.empty(p, dtype=torch.float64, device=dev),
                       lam=torch.empty(r, dtype=torch.float64, device=dev),
                       sure=torch.empty(r, dtype=torch.float64, device=dev),
                       gap=torch.empty(1, dtype=torch.float64, device=dev),
                       status=torch.zeros(1, dtype=torch.int32, device=dev),
                       rank=torch.zeros(1, dtype=torch.int32, device=dev))
            sg = None if sigmas is None or sigmas[i] is None else \
                sigmas[i].to(device=dev, dtype=torch.float64).contiguous()
            lm = None if lams is None or lams[i] is None else \
                lams[i].to(device=dev, dtype=torch.float64).contiguous()
            self._keep += [sg, lm]
            out = L.Outputs(inf["sigma"].data_ptr(), inf["V"].data_ptr(), inf["evals"].data_ptr(),
                            inf["lam"].data_ptr(), inf["sure"].data_ptr(), inf["gap"].data_ptr(),
                            inf["status"].data_ptr(), inf["rank"].data_ptr())
            xp, xrp = _cube_strides(X)
            arr[i] = L.Cube(Y.data_ptr(), H, W, p, pitch, rp, X.data_ptr(), xp, xrp, r, levels[i],
                            _ptr(sg), _ptr(lm), out)
            self.X.append(X)
            self._info.append(inf)
        self._cubes = arr
        lib = L.lib()
        nb = C.c_size_t()
        L.check(lib.hyres_batch_workspace_size(arr, count, self.dt, C.byref(self.opt), C.byref(nb)),
                "batch workspace size")
        self.ws_bytes = nb.value
        self._buf, self._ws = _workspace(nb.value, dev)
        self._h = _handle(dev)
        bp = C.c_void_p()
        L.check(lib.hyres_batch_create(self._h, arr, count, self.dt, C.byref(self.opt), self._ws, self.ws_bytes,
                                       _stream(dev), C.byref(bp)), "hyres_batch_create")
        self._b = bp.value

    def run(self):
        L.check(L.lib().hyres_batch_run(self._b, _stream(self.device)), "hyres_batch_run")
        return self.X

    def launch_graph(self):
        L.check(L.lib().hyres_batch_launch_graph(self._b, _stream(self.device)), "hyres_batch_launch_graph")
        return self.X

    def autotune(self, cache_path: Optional[str] = None):
        path = None if cache_path is None else cache_path.encode()
        L.check(L.lib().hyres_autotune(self._h, self._b, path, _stream(self.device)), "hyres_autotune")

    def info(self, i: int) -> Dict[str, torch.Tensor]:
        d = dict(self._info[i])
        d["V"] = d["V"].T
        return d

    def __del__(self):
        b = getattr(self, "_b", None)
        if b:
            try:
                L.lib().hyres_batch_destroy(b)
            except Exception:   # interpreter shutdown
                pass
            self._b = None


def denoise_batched(cubes, ranks, levels, precision: str = "native", scope: str = "all", graph: bool = False):
    """Denoise a list of cubes in one batched solve; returns [(X, info), ...]."""
    b = Batch(cubes, ranks, levels, precision=precision, scope=scope)
    if graph:
        b.launch_graph()
    else:
        b.run()
    return [(b.X[i], b.info(i)) for i in range(len(cubes))], b


def tile_choice(dtype: torch.dtype, inverse: bool, width: int, device=None):
    """(tx, ty, tuned) the handle uses for a transform level of this width."""
    dev = torch.device(device if device is not None else "cuda")
    tx, ty, tu = C.c_int(), C.c_int(), C.c_int()
    dt = L.HYRES_F64 if dtype == torch.float64 else L.HYRES_F32
    L.check(L.lib().hyres_tile_choice(_handle(dev), dt, int(inverse), int(width), C.byref(tx), C.byref(ty),
                                      C.byref(tu)), "hyres_tile_choice")
    return tx.value, ty.value, bool(tu.value)


def tile_grid(size: int, tile: int, overlap: int):
    """Tile starts along one axis (the library's rule)."""
    n = C.c_int()
    buf = (C.c_int * 64)()
    L.check(L.lib().hyres_tile_grid(size, tile, overlap, buf, C.byref(n)), "hyres_tile_grid")
    return [buf[i] for i in range(n.value)]


def denoise_tiled(Y: torch.Tensor, rank: int, levels: int, tile: int = 512, overlap: int = 32,
                  precision: str = "native", scope: str = "all", X: Optional[torch.Tensor] = None):
    """Sliding-window HyRes: every tile denoised independently, then blended.

    Returns (X, info) with info["lam"] of shape (tiles, rank), info["sigma"]
    (tiles, p) and the shared device status word.
    """
    _need_cuda(Y, "Y")
    H, W, p = Y.shape
    pitch, rp = _cube_strides(Y)
    dt = _dtype_code(Y)
    opt = L.Options(rank, levels, L.PREC_MIXED if precision == "mixed" else L.PREC_NATIVE,
                    L.SCOPE_ALL if scope == "all" else L.SCOPE_DETAIL, 0)
    lib = L.lib()
    nb = C.c_size_t()
    L.check(lib.hyres_tiled_workspace_size(H, W, p, tile, overlap, C.byref(opt), dt, C.byref(nb)),
            "tiled workspace size")
    buf, ws = _workspace(nb.value, Y.device)
    nt = len(tile_grid(H, tile, overlap)) * len(tile_grid(W, tile, overlap))
    lam = torch.empty(nt, rank, dtype=torch.float64, device=Y.device)
    sig = torch.empty(nt, p, dtype=torch.float64, device=Y.device)
    status = torch.zeros(1, dtype=torch.int32, device=Y.device)
    if X is None:
        X = torch.empty(H, W, p, dtype=Y.dtype, device=Y.device)
    xp, xrp = _cube_strides(X)
    L.check(lib.hyres_denoise_tiled(_handle(Y.device), Y.data_ptr(), H, W, p, pitch, rp, dt, tile, overlap,
                                    C.byref(opt), X.data_ptr(), xp, xrp, lam.data_ptr(), sig.data_ptr(),
                                    status.data_ptr(), ws, nb.value, _stream(Y.device)), "hyres_denoise_tiled")
    return X, dict(lam=lam, sigma=sig, status=status)


# ------------------------------------------------------------------ adjoint
def sure_grad(coeffs: torch.Tensor, lam: torch.Tensor) -> torch.Tensor:
    """d SURE / d lambda_i at lambda_i for each row of a (B, N) tensor."""
    _need_cuda(coeffs, "coeffs")
    if coeffs.stride(1) != 1:
        coeffs = coeffs.contiguous()
    B, N = coeffs.shape
    lib = L.lib()
    nb = C.c_size_t()
    L.check(lib.hyres_sure_grad_workspace_size(B, N, C.byref(nb)), "workspace size")
    buf, ws = _workspace(nb.value, coeffs.device)
    lm = lam.to(device=coeffs.device, dtype=torch.float64).contiguous()
    out = torch.empty(B, dtype=torch.float64, device=coeffs.device)
    row_stride = coeffs.stride(0) if B > 1 else N
    L.check(lib.hyres_sure_grad(_handle(coeffs.device), coeffs.data_ptr(), B, N, row_stride, _dtype_code(coeffs),
                                lm.data_ptr(), out.data_ptr(), ws, nb.value, _stream(coeffs.device)),
            "hyres_sure_grad")
    return out


def denoise_backward(dn: "Denoiser", Y: torch.Tensor, dX: torch.Tensor):
    """(dY, dlambda) of the solve last run by Denoiser ``dn`` on ``Y``."""
    dX = dX.contiguous()
    pitch, rp = _cube_strides(Y)
    xp, xrp = _cube_strides(dX)
    dY = torch.empty(dn.H, dn.W, dn.p, dtype=dn.dtype, device=dn.device)
    yp, yrp = _cube_strides(dY)
    dlam = torch.empty(dn.r, dtype=torch.float64, device=dn.device)
    status = torch.zeros(1, dtype=torch.int32, device=dn.device)
    lib = L.lib()
    nb = C.c_size_t()
    L.check(lib.hyres_denoise_backward_workspace_size(dn.H, dn.W, dn.p, C.byref(dn.opt), dn.dt, C.byref(nb)),
            "backward workspace size")
    buf, ws = _workspace(nb.value, dn.device)
    L.check(lib.hyres_denoise_backward(_handle(dn.device), Y.data_ptr(), dn.H, dn.W, dn.p, pitch, rp, dn.dt,
                                       C.byref(dn.opt), dn._ws, dn.ws_bytes, C.byref(dn.out), dX.data_ptr(), xp, xrp,
                                       dY.data_ptr(), yp, yrp, dlam.data_ptr(), status.data_ptr(), ws, nb.value,
                                       _stream(dn.device)), "hyres_denoise_backward")
    return dY, dlam, status


class HyResFunction(torch.autograd.Function):
    """X = HyRes(Y; lambda) with a hand-written adjoint.

    ``HyResFunction.apply(Y, lam, rank, levels, precision)``: lambda is a
    tensor of per-component thresholds (an input, so it gets a gradient).
    The forward keeps the solve's workspace (band Gram, coefficients and
    denoised component images) for the backward.
    """

    @staticmethod
    def forward(ctx, Y, lam, rank: int, levels: int, precision: str = "native"):
        _need_cuda(Y, "Y")
        H, W, p = Y.shape
        dn = Denoiser(H, W, p, rank, levels, dtype=Y.dtype, precision=precision, device=Y.device)
        lm = lam.detach().to(device=Y.device, dtype=torch.float64).contiguous()
        Yc = Y.detach()
        X = dn.run(Yc, None, lm).clone()
        ctx.dn = dn
        ctx.lam_keep = lm
        ctx.save_for_backward(Yc)
        ctx.lam_meta = (lam.dtype, lam.device)
        return X

    @staticmethod
    def backward(ctx, dX):
        (Y,) = ctx.saved_tensors
        dY, dlam, status = denoise_backward(ctx.dn, Y, dX)
        dt, dev = ctx.lam_meta
        return dY, dlam.to(device=dev, dtype=dt), None, None, None
