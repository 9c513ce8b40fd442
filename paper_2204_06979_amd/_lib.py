"""ctypes declarations of libhyres.so (the C ABI in include/hyres.h).

Argument marshalling only: every step of the denoiser runs in the library's
HIP kernels.  Importing this module fails loudly when the library has not
been built; there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhyres.so")

HYRES_OK = 0
STATUS_NAMES = {0: "HYRES_OK", 1: "HYRES_E_NULL", 2: "HYRES_E_SHAPE", 3: "HYRES_E_DTYPE",
                4: "HYRES_E_WORKSPACE", 5: "HYRES_E_HIP", 6: "HYRES_E_UNSUPPORTED"}
HYRES_F32, HYRES_F64 = 0, 1
PREC_NATIVE, PREC_MIXED = 0, 1
SCOPE_ALL, SCOPE_DETAIL = 0, 1
DEV_NOT_PD, DEV_NONFINITE, DEV_EIGH_NOCONV, DEV_DEGENERATE, DEV_SURE_INEXACT = 1, 2, 4, 8, 16


FLAG_ALL_EVALS = 1
FLAG_RANK_HYSIME, FLAG_RANK_SURE = 2, 4
NOALLOC_SCRATCH_BYTES = 96 << 20     # HYRES_NOALLOC_SCRATCH_BYTES


class Options(C.Structure):
    _fields_ = [("rank", C.c_int), ("levels", C.c_int), ("precision", C.c_int), ("scope", C.c_int),
                ("flags", C.c_int)]


class Outputs(C.Structure):
    _fields_ = [("sigma", C.c_void_p), ("V", C.c_void_p), ("evals", C.c_void_p), ("lambda_", C.c_void_p),
                ("sure", C.c_void_p), ("gap", C.c_void_p), ("status", C.c_void_p), ("rank", C.c_void_p),
                ("eig_check", C.c_void_p)]


class L1Options(C.Structure):
    _fields_ = [("lam", C.c_double), ("mu1", C.c_double), ("mu2", C.c_double), ("iters", C.c_int)]


class Cube(C.Structure):
    _fields_ = [("Y", C.c_void_p), ("H", C.c_int), ("W", C.c_int), ("p", C.c_int), ("pitch", C.c_int64),
                ("row_pitch", C.c_int64), ("X", C.c_void_p), ("x_pitch", C.c_int64), ("x_row_pitch", C.c_int64),
                ("rank", C.c_int), ("levels", C.c_int), ("sigma_in", C.c_void_p), ("lambda_in", C.c_void_p),
                ("out", Outputs)]


class ProgramStats(C.Structure):
    _fields_ = [("launches", C.c_int), ("records", C.c_int), ("waits", C.c_int), ("streams", C.c_int),
                ("groups", C.c_int)]


vp, i32, i64, sz, dp = C.c_void_p, C.c_int, C.c_int64, C.c_size_t, C.c_void_p
PI = C.POINTER(C.c_int)

# name -> (restype, argtypes)
SIGNATURES = {
    "hyres_create": (i32, [C.POINTER(C.c_void_p), i32]),
    "hyres_destroy": (None, [vp]),
    "hyres_status_string": (C.c_char_p, [i32]),
    "hyres_coeff_count": (i64, [i32, i32, i32]),
    "hyres_estimate_noise_workspace_size": (i32, [i32, i32, i32, i32, C.POINTER(sz)]),
    "hyres_estimate_noise": (i32, [vp, vp, i32, i32, i32, i64, i64, i32, dp, dp, vp, vp, sz, vp]),
    "hyres_subspace_workspace_size": (i32, [i32, i32, i32, i32, i32, C.POINTER(sz)]),
    "hyres_subspace": (i32, [vp, vp, i32, i32, i32, i64, i64, i32, dp, i32, dp, dp, vp, vp, sz, vp]),
    "hyres_dwt2_workspace_size": (i32, [i32, i32, i32, i32, i32, C.POINTER(sz)]),
    "hyres_dwt2": (i32, [vp, vp, i32, i32, i32, i32, i32, vp, vp, sz, vp]),
    "hyres_idwt2": (i32, [vp, vp, i32, i32, i32, i32, i32, dp, i32, vp, vp, sz, vp]),
    "hyres_sure_workspace_size": (i32, [i32, i64, i32, C.POINTER(sz)]),
    "hyres_sure_threshold": (i32, [vp, vp, i32, i64, i64, i32, dp, dp, vp, vp, sz, vp]),
    "hyres_denoise_workspace_size": (i32, [i32, i32, i32, C.POINTER(Options), i32, C.POINTER(sz)]),
    "hyres_profile_enable": (i32, [vp, C.c_uint]),
    "hyres_profile_read": (i32, [vp, C.POINTER(C.c_double), C.POINTER(C.c_int)]),
    "hyres_denoise": (i32, [vp, vp, i32, i32, i32, i64, i64, i32, C.POINTER(Options), dp, dp, vp, i64, i64,
                            C.POINTER(Outputs), vp, sz, vp]),
    "hyres_l1l1_spectral": (i32, [vp, vp, i32, i32, i32, i64, i64, i32, C.POINTER(L1Options), vp, i64, i64, vp]),
    "hyres_hyminor": (i32, [vp, vp, i32, i32, i32, i64, i64, i32, C.POINTER(Options), dp, dp,
                            C.POINTER(L1Options), vp, i64, i64, C.POINTER(Outputs), vp, sz, vp]),
    "hyres_wsrrr_workspace_size": (i32, [i32, i32, i32, C.POINTER(Options), i32, C.POINTER(sz)]),
    "hyres_wsrrr": (i32, [vp, vp, i32, i32, i32, i64, i64, i32, C.POINTER(Options), i32, dp, dp, vp, i64, i64,
                          C.POINTER(Outputs), vp, sz, vp]),
    "hyres_forpdn_workspace_size": (i32, [i32, i32, i32, i32, i32, i32, C.POINTER(sz)]),
    "hyres_forpdn": (i32, [vp, vp, i32, i32, i32, i64, i64, i32, i32, dp, dp, vp, i64, i64, dp, dp, dp, vp, vp,
                           sz, vp]),
    "hyres_denoise_noalloc": (i32, [vp, vp, i32, i32, i32, i64, i64, i32, C.POINTER(Options), dp, dp, vp, i64,
                                    i64, C.POINTER(Outputs), vp]),
    "hyres_batch_workspace_size": (i32, [C.POINTER(Cube), i32, i32, C.POINTER(Options), C.POINTER(sz)]),
    "hyres_batch_create": (i32, [vp, C.POINTER(Cube), i32, i32, C.POINTER(Options), vp, sz, vp,
                                 C.POINTER(C.c_void_p)]),
    "hyres_batch_run": (i32, [vp, vp]),
    "hyres_batch_launch_graph": (i32, [vp, vp]),
    "hyres_batch_destroy": (None, [vp]),
    "hyres_denoise_batched": (i32, [vp, C.POINTER(Cube), i32, i32, C.POINTER(Options), vp, sz, vp]),
    "hyres_autotune": (i32, [vp, vp, C.c_char_p, vp]),
    "hyres_tile_choice": (i32, [vp, i32, i32, i32, PI, PI, PI]),
    "hyres_tile_grid": (i32, [i32, i32, i32, PI, PI]),
    "hyres_tiled_workspace_size": (i32, [i32, i32, i32, i32, i32, C.POINTER(Options), i32, C.POINTER(sz)]),
    "hyres_denoise_tiled": (i32, [vp, vp, i32, i32, i32, i64, i64, i32, i32, i32, C.POINTER(Options), vp, i64,
                                  i64, dp, dp, vp, vp, sz, vp]),
    "hyres_denoise_backward_workspace_size": (i32, [i32, i32, i32, C.POINTER(Options), i32, C.POINTER(sz)]),
    "hyres_denoise_backward": (i32, [vp, vp, i32, i32, i32, i64, i64, i32, C.POINTER(Options), vp, sz,
                                     C.POINTER(Outputs), vp, i64, i64, vp, i64, i64, dp, vp, vp, sz, vp]),
    "hyres_sure_grad_workspace_size": (i32, [i32, i64, C.POINTER(sz)]),
    "hyres_sure_grad": (i32, [vp, vp, i32, i64, i64, i32, dp, dp, vp, sz, vp]),
    "hyres_batch_check_program": (i32, [C.POINTER(Cube), i32, i32, C.POINTER(Options), C.POINTER(ProgramStats)]),
    "hyres_tiled_check_program": (i32, [i32, i32, i32, i32, i32, C.POINTER(Options), i32,
                                        C.POINTER(ProgramStats)]),
}


def load(path: str = LIB_PATH) -> C.CDLL:
    if not os.path.exists(path):
        raise ImportError("libhyres.so is not built at %s; run `python -m paper_2204_06979_amd.build`" % path)
    lib = C.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


_LIB = None


def lib() -> C.CDLL:
    global _LIB
    if _LIB is None:
        _LIB = load()
    return _LIB


class HyresError(RuntimeError):
    pass


def check(status: int, what: str = "") -> None:
    if status != HYRES_OK:
        msg = lib().hyres_status_string(status).decode()
        raise HyresError("%s failed: %s (%s)" % (what, STATUS_NAMES.get(status, status), msg))
