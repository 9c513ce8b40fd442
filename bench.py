#!/usr/bin/env python3
"""HyRes solve throughput on one MI355X.

Workload: a synthetic 349 x 1905 x 144 FP32 cube (the shape of the Houston
2013 scene the paper evaluates on), rank 8, 4 wavelet levels, per-band SNR
drawn in 5-20 dB.  One step = one complete HyRes solve (noise estimate,
eigensolve, projection, transforms, SURE thresholds, inverse, back-projection)
with the cube already resident in HBM.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import ctypes as C
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "denoised voxels/s per HyRes solve, mixed vs FP32, at stated err; HBM GB/s"
STAGES = ["gram", "small", "project", "dwt", "sure", "idwt", "backproject"]
HBM_PEAK_GBS = 8000.0
PEAK_TFLOPS = {"native": 157.3, "mixed": 2500.0}    # FP32 matrix / BF16 dense matrix


def stage_work(H, W, p, r, L):
    """Algorithmic bytes (or flops) of one launch of each stage, FP32 elements.

    SURE is charged two reads of the coefficients (one histogram pass and one
    refinement pass), whatever number of refinement rounds the kernels run."""
    from paper_2204_06979_amd.api import coeff_count
    n = H * W
    s = 4
    nc = coeff_count(H, W, L)
    return {
        "gram": ("mfma", float(n) * p * (p + 1), "TFLOP/s"),
        "project": ("hbm", float(s) * (n * p + n * r), "GB/s"),
        "dwt": ("hbm", float(s) * r * (n + nc), "GB/s"),
        "sure": ("hbm", float(s) * r * nc * 2, "GB/s"),
        "idwt": ("hbm", float(s) * r * (nc + n), "GB/s"),
        "backproject": ("hbm", float(s) * (n * r + n * p), "GB/s"),
    }


def measure(api, _lib, lib, handle, Y, dims, precision, steps, warmup):
    """Warm up, take a per-stage breakdown, then time `steps` solves with HIP
    events around the dominant stage (on the solve stream)."""
    import torch
    H, W, p, r, L = dims
    dev = Y.device
    dn = api.Denoiser(H, W, p, r, L, dtype=torch.float32, precision=precision, device=dev)
    for _ in range(max(warmup, 1)):
        dn.run(Y)
    torch.cuda.synchronize()
    ms = (C.c_double * 7)()
    cnt = (C.c_int * 7)()
    lib.hyres_profile_enable(handle, (1 << len(STAGES)) - 1)
    for _ in range(3):
        dn.run(Y)
    torch.cuda.synchronize()
    _lib.check(lib.hyres_profile_read(handle, ms, cnt), "profile read")
    stage_ms = {STAGES[i]: ms[i] / max(cnt[i], 1) for i in range(7)}
    work = stage_work(H, W, p, r, L)
    dom = max(work.keys(), key=lambda k: stage_ms[k])
    dom_bit = STAGES.index(dom)
    for i in range(7):
        ms[i] = 0.0
        cnt[i] = 0
    lib.hyres_profile_enable(handle, 1 << dom_bit)
    stream = torch.cuda.current_stream(dev)
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    ev0.record(stream)
    for _ in range(steps):
        dn.run(Y)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    _lib.check(lib.hyres_profile_read(handle, ms, cnt), "profile read")
    lib.hyres_profile_enable(handle, 0)
    ms_step = ev0.elapsed_time(ev1) / steps
    dom_ms = ms[dom_bit] / max(cnt[dom_bit], 1)
    bound, amount, unit = work[dom]
    if bound == "mfma":
        achieved = amount / (dom_ms * 1e-3) / 1e12
        peak = PEAK_TFLOPS[precision]
    else:
        achieved = amount / (dom_ms * 1e-3) / 1e9
        peak = HBM_PEAK_GBS
    return dict(dn=dn, ms_step=ms_step, wall=wall, stage_ms=stage_ms, dom=dom, dom_ms=dom_ms,
                roofline={"bound": bound, "kernel": dom, "achieved": achieved, "peak": peak, "unit": unit,
                          "frac": achieved / peak, "traffic": None, "kernel_ms": dom_ms},
                status=int(dn.status.cpu()[0]))


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--precision", default="both", choices=["native", "mixed", "both"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-parity", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this build runs the HyRes path on one GPU only; --gpus %d is not supported"
              % args.gpus, file=sys.stderr)
        return 2

    import torch
    from paper_2204_06979_amd import _lib, api, synth

    cfg = synth.CONFIG_SHAPES[2]
    H, W, p, r, L = cfg["H"], cfg["W"], cfg["p"], cfg["r"], cfg["levels"]
    t0 = time.time()
    cube = synth.config_cube(2, keep_clean=False)
    print("bench: generated %dx%dx%d cube in %.1f s" % (H, W, p, time.time() - t0), file=sys.stderr, flush=True)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    Y = torch.tensor(cube.Y, device=dev)
    lib = _lib.lib()
    handle = api._handle(dev)
    precs = ["native", "mixed"] if args.precision == "both" else [args.precision]
    res = {}
    for prec in precs:
        res[prec] = measure(api, _lib, lib, handle, Y, (H, W, p, r, L), prec, args.steps, args.warmup)
        print("bench: %s %.3f ms/solve" % (prec, res[prec]["ms_step"]), file=sys.stderr, flush=True)
    head = res["mixed"] if "mixed" in res else res[precs[0]]
    head_prec = "mixed" if "mixed" in res else precs[0]
    voxels = float(H * W * p)
    out = {
        "metric": METRIC,
        "value": voxels / (head["ms_step"] * 1e-3),
        "unit": "voxels/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16-split/f32" if head_prec == "mixed" else "f32",
        "data": "synthetic",
        "config": {
            "workload": "HyRes solve of a %dx%dx%d FP32 cube (Houston-2013 shape), rank %d, %d db2 levels, "
                        "per-band SNR 5-20 dB, linear-mixing synthetic" % (H, W, p, r, L),
            "precision": head_prec,
        },
        "roofline": head["roofline"],
    }
    for prec, m in res.items():
        out["config"][prec] = {"voxels_per_s": voxels / (m["ms_step"] * 1e-3), "ms_per_solve": m["ms_step"],
                               "wall_s": m["wall"], "stages_ms": m["stage_ms"], "roofline": m["roofline"],
                               "hbm_gbs_whole_solve": (4.0 * (3 * H * W * p)) / (m["ms_step"] * 1e-3) / 1e9,
                               "device_status": m["status"]}

    if not args.no_parity or not args.no_cpu_baseline:
        from oracle import hyres_oracle as O
        try:
            from threadpoolctl import threadpool_info
            cores = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
        except Exception:  # pragma: no cover
            cores = len(os.sched_getaffinity(0))
        c0 = time.perf_counter()
        ref = O.hyres(cube.Y.astype(np.float64), r, L)
        cpu_s = time.perf_counter() - c0
        for prec, m in res.items():
            X = m["dn"].run(Y).double().cpu().numpy()
            err = float(np.linalg.norm(X - ref["X"]) / np.linalg.norm(ref["X"]))
            dn = m["dn"]
            out["config"][prec]["rel_err_vs_fp64_oracle"] = err
            out["config"][prec]["sigma_max_rel_err"] = float(np.max(np.abs(dn.sigma.cpu().numpy() / ref["sigma"] - 1)))
            out["config"][prec]["evals_top_r_max_rel_err"] = float(np.max(np.abs(
                dn.evals.cpu().numpy()[:r] / ref["evals"][:r] - 1)))
            out["config"][prec]["lambda_max_rel_diff"] = float(np.max(np.abs(dn.lam.cpu().numpy() - ref["lam"])
                                                                   / ref["lam"]))
        if not args.no_cpu_baseline:
            out["cpu_baseline"] = {"value": voxels / cpu_s, "unit": "voxels/s", "cores": int(cores),
                                   "kind": "oracle",
                                   "sample": "one full oracle solve of the same %dx%dx%d cube (FP64 numpy), "
                                             "%.1f s" % (H, W, p, cpu_s)}
    print(json.dumps(out))
    return 0


if __name__ == "__main__":
    sys.exit(main())
