#!/usr/bin/env python3
"""HyRes solve throughput on one MI355X.

Default workload: a synthetic 349 x 1905 x 144 FP32 cube (the shape of the
Houston 2013 scene the paper evaluates on), rank 8, 4 wavelet levels,
per-band SNR drawn in 5-20 dB.  One step = one complete HyRes solve (noise
estimate, eigensolve, projection, transforms, SURE thresholds, inverse,
back-projection) with the cube already resident in HBM.  Prints one JSON line.

``--workload batch`` times the 64-cube batch (uneven sizes, one HIP graph
replay per step, DWT tiles autotuned first) and ``--workload tiled`` the
2048 x 2048 x 224 sliding-window solve (25 tiles of 512^2, 32 px overlap);
both print the same JSON contract for their workload.
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
FP64_VECTOR_TFLOPS = 78.6
PEAK_TFLOPS = {"native": 157.3, "mixed": 2500.0}    # FP32 matrix / BF16 dense matrix
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")


def stage_work(shapes, precision):
    """Algorithmic work of one launch sequence of each stage over the cubes
    ``shapes`` = [(H, W, p, r, L), ...] (FP32 elements).

    gram: n p (p + 1) flops (upper triangle of the SYRK, as two flops per MAC);
    small: FP64 flops of the sweep (2 p^3), the Householder reduction
    (4/3 p^3) and the back-transform of r + 1 vectors (2 p^2 (r + 1));
    project/backproject: the cube once plus the r component images;
    dwt/idwt: the component images plus the coefficients;
    sure: two reads of the coefficients (histogram pass and refinement pass),
    whatever number of refinement rounds the kernels run.
    """
    from paper_2204_06979_amd.api import coeff_count
    w = {k: 0.0 for k in STAGES}
    for (H, W, p, r, L) in shapes:
        n = H * W
        nc = coeff_count(H, W, L)
        w["gram"] += float(n) * p * (p + 1)
        w["small"] += 2.0 * p ** 3 + 4.0 / 3.0 * p ** 3 + 2.0 * p * p * (r + 1)
        w["project"] += 4.0 * (n * p + n * r)
        w["dwt"] += 4.0 * r * (n + nc)
        w["sure"] += 4.0 * r * nc * 2
        w["idwt"] += 4.0 * r * (nc + n)
        w["backproject"] += 4.0 * (n * r + n * p)
    kinds = {"gram": ("mfma", PEAK_TFLOPS[precision], "TFLOP/s"),
             "small": ("alu", FP64_VECTOR_TFLOPS, "TFLOP/s")}
    out = {}
    for k in STAGES:
        bound, peak, unit = kinds.get(k, ("hbm", HBM_PEAK_GBS, "GB/s"))
        out[k] = (bound, w[k], peak, unit)
    return out


def roofline_of(stage, work, ms, traffic):
    bound, amount, peak, unit = work[stage]
    scale = 1e12 if unit == "TFLOP/s" else 1e9
    achieved = amount / (ms * 1e-3) / scale
    return {"bound": bound, "kernel": stage, "achieved": achieved, "peak": peak, "unit": unit,
            "frac": achieved / peak, "traffic": traffic, "kernel_ms": ms}


def load_traffic(workload, stage):
    """HBM bytes per launch sequence of `stage` from the committed counter summary, if it covers
    this workload and stage."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
        e = t.get(workload, {}).get(stage)
        return None if e is None else e.get("bytes")
    except (OSError, ValueError):
        return None


class Timer:
    """Per-stage times through the library's stage timers (HIP events on the solve stream)."""

    def __init__(self, _lib, lib, handle):
        self._lib, self.lib, self.h = _lib, lib, handle

    def stages(self, run, reps=3, mask=None):
        import torch
        ms = (C.c_double * 7)()
        cnt = (C.c_int * 7)()
        self.lib.hyres_profile_enable(self.h, (1 << len(STAGES)) - 1 if mask is None else mask)
        for _ in range(reps):
            run()
        torch.cuda.synchronize()
        self._lib.check(self.lib.hyres_profile_read(self.h, ms, cnt), "profile read")
        self.lib.hyres_profile_enable(self.h, 0)
        return {STAGES[i]: ms[i] / max(cnt[i], 1) for i in range(7) if cnt[i]}


def timed_steps(run, steps, dom_bit, timer):
    """Time `steps` runs with events on the current stream; the dominant stage
    is timed at the same time by the library's stage timers."""
    import torch
    stream = torch.cuda.current_stream()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ms = (C.c_double * 7)()
    cnt = (C.c_int * 7)()
    if dom_bit is not None:
        timer.lib.hyres_profile_enable(timer.h, 1 << dom_bit)
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    ev0.record(stream)
    for _ in range(steps):
        run()
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    dom_ms = None
    if dom_bit is not None:
        timer._lib.check(timer.lib.hyres_profile_read(timer.h, ms, cnt), "profile read")
        timer.lib.hyres_profile_enable(timer.h, 0)
        dom_ms = ms[dom_bit] / max(cnt[dom_bit], 1)
    return ev0.elapsed_time(ev1) / steps, wall, dom_ms


def measure_single(api, timer, Y, dims, precision, steps, warmup, workload):
    import torch
    H, W, p, r, L = dims
    dn = api.Denoiser(H, W, p, r, L, dtype=torch.float32, precision=precision, device=Y.device)
    for _ in range(max(warmup, 1)):
        dn.run(Y)
    torch.cuda.synchronize()
    stage_ms = timer.stages(lambda: dn.run(Y))
    work = stage_work([dims], precision)
    dom = max(stage_ms, key=lambda k: stage_ms[k])
    ms_step, wall, dom_ms = timed_steps(lambda: dn.run(Y), steps, STAGES.index(dom), timer)
    rl = {k: roofline_of(k, work, stage_ms[k], None) for k in stage_ms}
    return dict(dn=dn, ms_step=ms_step, wall=wall, stage_ms=stage_ms, dom=dom,
                roofline=roofline_of(dom, work, dom_ms, load_traffic(workload + "/" + precision, dom)),
                stage_rooflines=rl, status=int(dn.status.cpu()[0]))


def parity_single(api, cube, Y, dims, res):
    from oracle import hyres_oracle as O
    H, W, p, r, L = dims
    c0 = time.perf_counter()
    ref = O.hyres(cube.Y.astype(np.float64), r, L)
    cpu_s = time.perf_counter() - c0
    for prec, m in res.items():
        dn = m["dn"]
        X = dn.run(Y).double().cpu().numpy()
        V = dn.V.T.cpu().numpy()
        cosines = np.linalg.svd(V.T @ ref["V"], compute_uv=False)
        m["errors"] = {
            "X_rel": float(np.linalg.norm(X - ref["X"]) / np.linalg.norm(ref["X"])),
            "sigma_max_rel": float(np.max(np.abs(dn.sigma.cpu().numpy() / ref["sigma"] - 1))),
            "evals_top_r_max_rel": float(np.max(np.abs(dn.evals.cpu().numpy()[:r] / ref["evals"][:r] - 1))),
            "subspace_max_angle_rad": float(np.arccos(np.clip(cosines.min(), -1.0, 1.0))),
            "V_max_abs_diff": float(np.max(np.abs(V - ref["V"]))),
            "lambda_max_rel_diff": float(np.max(np.abs(dn.lam.cpu().numpy() - ref["lam"]) / ref["lam"])),
        }
    return cpu_s


def cpu_cores():
    try:
        from threadpoolctl import threadpool_info
        return max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:  # pragma: no cover
        return len(os.sched_getaffinity(0))


def run_single(args, api, timer, synth):
    import torch
    cfg = synth.CONFIG_SHAPES[2]
    dims = (cfg["H"], cfg["W"], cfg["p"], cfg["r"], cfg["levels"])
    H, W, p, r, L = dims
    t0 = time.time()
    cube = synth.config_cube(2, keep_clean=False)
    print("bench: generated %dx%dx%d cube in %.1f s" % (H, W, p, time.time() - t0), file=sys.stderr, flush=True)
    Y = torch.tensor(cube.Y, device="cuda")
    precs = ["native", "mixed"] if args.precision == "both" else [args.precision]
    res = {}
    for prec in precs:
        res[prec] = measure_single(api, timer, Y, dims, prec, args.steps, args.warmup, "single")
        print("bench: %s %.3f ms/solve" % (prec, res[prec]["ms_step"]), file=sys.stderr, flush=True)
    cpu_s = None
    if not args.no_parity or not args.no_cpu_baseline:
        cpu_s = parity_single(api, cube, Y, dims, res)
    workload = ("HyRes solve of a %dx%dx%d FP32 cube (Houston-2013 shape), rank %d, %d db2 levels, "
                "per-band SNR 5-20 dB, linear-mixing synthetic" % dims)
    sample = "one full oracle solve of the same %dx%dx%d cube (FP64 numpy)" % (H, W, p)
    return res, float(H * W * p), workload, cpu_s, sample


def run_batch(args, api, timer, synth):
    import torch
    t0 = time.time()
    cubes = synth.config3_cubes()
    print("bench: generated %d cubes in %.1f s" % (len(cubes), time.time() - t0), file=sys.stderr, flush=True)
    Yt = [torch.tensor(c.Y, device="cuda") for c in cubes]
    shapes = [(c.Y.shape[0], c.Y.shape[1], c.Y.shape[2], c.rank, c.levels) for c in cubes]
    precs = ["native", "mixed"] if args.precision == "both" else [args.precision]
    res = {}
    for prec in precs:
        b = api.Batch(Yt, [c.rank for c in cubes], [c.levels for c in cubes], precision=prec)
        b.run()
        b.autotune(os.path.join(ROOT, "gpurun_out", "dwt_tiles.json") if args.tune_cache is None
                   else args.tune_cache)
        for _ in range(max(args.warmup, 1)):
            b.launch_graph()
        torch.cuda.synchronize()
        stage_ms = timer.stages(b.run)
        work = stage_work(shapes, prec)
        dom = max(stage_ms, key=lambda k: stage_ms[k])
        ms_step, wall, _ = timed_steps(b.launch_graph, args.steps, None, timer)
        _, _, dom_ms = timed_steps(b.run, 3, STAGES.index(dom), timer)
        status = max(int(b.info(i)["status"].cpu()[0]) for i in range(len(cubes)))
        res[prec] = dict(batch=b, ms_step=ms_step, wall=wall, stage_ms=stage_ms, dom=dom,
                         roofline=roofline_of(dom, work, dom_ms, load_traffic("batch/" + prec, dom)),
                         stage_rooflines={k: roofline_of(k, work, stage_ms[k], None) for k in stage_ms},
                         status=status)
        print("bench: batch %s %.3f ms/step (graph)" % (prec, ms_step), file=sys.stderr, flush=True)
    cpu_s = None
    sample = None
    if not args.no_parity or not args.no_cpu_baseline:
        from oracle import hyres_oracle as O
        # the oracle on the smallest cubes of the batch, scaled by voxels
        order = sorted(range(len(cubes)), key=lambda i: cubes[i].Y.size)[:4]
        c0 = time.perf_counter()
        vox = 0
        refs = {}
        for i in order:
            c = cubes[i]
            refs[i] = O.hyres(c.Y.astype(np.float64), c.rank, c.levels)
            vox += c.Y.size
        cpu_s = (time.perf_counter() - c0) * sum(c.Y.size for c in cubes) / vox
        sample = "oracle solves of the 4 smallest of the 64 cubes (%d voxels), scaled to the batch" % vox
        for prec, m in res.items():
            b = m["batch"]
            errs = []
            for i in order:
                X = b.X[i].double().cpu().numpy()
                errs.append(float(np.linalg.norm(X - refs[i]["X"]) / np.linalg.norm(refs[i]["X"])))
            m["errors"] = {"X_rel_max_over_sampled_cubes": max(errs)}
    total = float(sum(c.Y.size for c in cubes))
    workload = ("batched HyRes of 64 uneven FP32 cubes (H, W in [128, 512], p in {103, 128, 191, 224}, "
                "rank 4-12, 4 db2 levels, 10 dB), one HIP graph replay per step, %.3f G voxels" % (total / 1e9))
    return res, total, workload, cpu_s, sample


def run_tiled(args, api, timer, synth):
    import torch
    t0 = time.time()
    cube = synth.config_cube(5, keep_clean=False)
    H, W, p = cube.Y.shape
    r, L, tile, ov = 10, 4, 512, 32
    print("bench: generated %dx%dx%d cube in %.1f s" % (H, W, p, time.time() - t0), file=sys.stderr, flush=True)
    Y = torch.tensor(cube.Y, device="cuda")
    del cube
    X = torch.empty_like(Y)
    starts_y, starts_x = api.tile_grid(H, tile, ov), api.tile_grid(W, tile, ov)
    shapes = [(tile, tile, p, r, L)] * (len(starts_y) * len(starts_x))
    precs = ["native", "mixed"] if args.precision == "both" else [args.precision]
    res = {}
    for prec in precs:
        run = lambda: api.denoise_tiled(Y, r, L, tile=tile, overlap=ov, precision=prec, X=X)   # noqa: E731
        for _ in range(max(args.warmup, 1)):
            _, info = run()
        torch.cuda.synchronize()
        stage_ms = timer.stages(run)
        work = stage_work(shapes, prec)
        dom = max(stage_ms, key=lambda k: stage_ms[k])
        ms_step, wall, dom_ms = timed_steps(run, args.steps, STAGES.index(dom), timer)
        res[prec] = dict(ms_step=ms_step, wall=wall, stage_ms=stage_ms, dom=dom,
                         roofline=roofline_of(dom, work, dom_ms, load_traffic("tiled/" + prec, dom)),
                         stage_rooflines={k: roofline_of(k, work, stage_ms[k], None) for k in stage_ms},
                         status=int(info["status"].cpu()[0]))
        print("bench: tiled %s %.3f ms/step" % (prec, ms_step), file=sys.stderr, flush=True)
    cpu_s = None
    sample = None
    if not args.no_cpu_baseline:
        from oracle import hyres_oracle as O
        sub = Y[:tile, :tile].cpu().numpy().astype(np.float64)
        c0 = time.perf_counter()
        O.hyres(sub, r, L)
        cpu_s = (time.perf_counter() - c0) * len(shapes) * H * W / (len(shapes) * tile * tile)
        sample = "oracle solve of one 512x512x224 tile, scaled to the 25 tiles (blend not timed)"
    workload = ("sliding-window HyRes of a %dx%dx%d FP32 cube, 25 tiles of 512x512 with 32 px overlap, "
                "rank 10, 4 db2 levels, SNR 5-15 dB + dead columns + 1%% impulses" % (H, W, p))
    return res, float(H * W * p), workload, cpu_s, sample


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--precision", default="both", choices=["native", "mixed", "both"])
    ap.add_argument("--workload", default="single", choices=["single", "batch", "tiled"])
    ap.add_argument("--tune-cache", default=None)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-parity", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this build runs the HyRes path on one GPU only; --gpus %d is not supported"
              % args.gpus, file=sys.stderr)
        return 2

    import torch
    from paper_2204_06979_amd import _lib, api, synth

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    lib = _lib.lib()
    timer = Timer(_lib, lib, api._handle(dev))
    runner = {"single": run_single, "batch": run_batch, "tiled": run_tiled}[args.workload]
    res, voxels, workload, cpu_s, sample = runner(args, api, timer, synth)
    head_prec = "mixed" if "mixed" in res else next(iter(res))
    head = res[head_prec]
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
        "config": {"workload": workload, "precision": head_prec},
        "roofline": head["roofline"],
    }
    for prec, m in res.items():
        e = {"voxels_per_s": voxels / (m["ms_step"] * 1e-3), "ms_per_step": m["ms_step"], "wall_s": m["wall"],
             "stages_ms": m["stage_ms"], "roofline": m["roofline"], "stage_rooflines": m["stage_rooflines"],
             "device_status": m["status"]}
        if "errors" in m:
            e["errors_vs_fp64_oracle"] = m["errors"]
        out["config"][prec] = e
    if cpu_s is not None and not args.no_cpu_baseline:
        out["cpu_baseline"] = {"value": voxels / cpu_s, "unit": "voxels/s", "cores": int(cpu_cores()),
                               "kind": "oracle", "sample": "%s, %.1f s" % (sample, cpu_s)}
    print(json.dumps(out))
    return 0


if __name__ == "__main__":
    sys.exit(main())
