#!/usr/bin/env python3
"""HyRes solve throughput on one MI355X.

Headline workload: a synthetic 349 x 1905 x 144 FP32 cube (the shape of the
Houston 2013 scene the paper evaluates on), rank 8, 4 wavelet levels,
per-band SNR drawn in 5-20 dB.  One step = one complete HyRes solve (noise
estimate, eigensolve, projection, transforms, SURE thresholds, inverse,
back-projection) with the cube already resident in HBM.  Two copies of the
cube are resident and the steps alternate between them, so no step reads a
cube that the previous step left in the last-level cache.

Every step is bracketed by its own pair of HIP events on the solve stream: the
line's ms_per_step is the mean over the K timed steps, and the paper's Olympic
score (fastest and slowest dropped, mean of the rest) is reported beside it
with the spread of the kept steps.

By default the line also carries, under config.workloads, the other
workloads: the 64 x 64 x 32 FP64 cube (rank 4, 3 levels), the 256 x 256 x 191
forward + backward (rank 6), the batch of 64 uneven cubes (one HIP graph
replay per step) and the 2048 x 2048 x 224 sliding window (25 tiles of 512^2,
32 px overlap), each with its rate, whole-solve algorithmic HBM bandwidth and
its error against the FP64 oracle.  ``--workload single|small|grad|batch|tiled``
runs one workload alone (the profiled runs use ``single``).
"""
from __future__ import annotations

import argparse
import ctypes as C
import json
import os
import platform
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


def log(*a):
    print("bench:", *a, file=sys.stderr, flush=True)


# ------------------------------------------------------------- work counts
def solve_bytes(shapes, elem=4, blended_output=None):
    """Algorithmic HBM bytes of one solve of the cubes ``shapes`` = [(H, W, p, r, L)]:
    the cube read twice (Gram pass, projection pass) and the output written
    once, plus per component the image written and read, the coefficients
    written, read by the threshold search and read by the inverse, and the
    denoised image written and read.  Intermediate transform levels are not
    counted (they can be fused away).  ``blended_output`` = (H, W, p): a
    sliding window writes one blended output instead of one per tile."""
    from paper_2204_06979_amd.api import coeff_count
    b = 0.0
    for (H, W, p, r, L) in shapes:
        n = H * W
        nc = coeff_count(H, W, L)
        out = 0 if blended_output else n * p
        b += elem * (2.0 * n * p + out) + elem * r * (4.0 * n + 3.0 * nc)
    if blended_output:
        H, W, p = blended_output
        b += elem * float(H) * W * p
    return b


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
    this workload and stage (entries are removed when their kernels change)."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
        e = t.get(workload, {}).get(stage)
        return None if e is None else e.get("bytes")
    except (OSError, ValueError):
        return None


# ------------------------------------------------------------------ timing
class Timer:
    """Per-stage times through the library's stage timers (HIP events on the solve stream)."""

    def __init__(self, _lib, lib, handle):
        self._lib, self.lib, self.h = _lib, lib, handle

    def stages(self, run, reps=3, mask=None):
        import torch
        ms = (C.c_double * 7)()
        cnt = (C.c_int * 7)()
        self.lib.hyres_profile_enable(self.h, (1 << len(STAGES)) - 1 if mask is None else mask)
        for i in range(reps):
            run(i)
        torch.cuda.synchronize()
        self._lib.check(self.lib.hyres_profile_read(self.h, ms, cnt), "profile read")
        self.lib.hyres_profile_enable(self.h, 0)
        return {STAGES[i]: ms[i] / max(cnt[i], 1) for i in range(7) if cnt[i]}


def olympic(per_step):
    """The paper's scoring: drop the fastest and the slowest run, mean of the rest."""
    a = sorted(per_step)
    kept = a[1:-1] if len(a) >= 3 else a
    return {"mean_ms": float(np.mean(kept)), "min_ms": float(kept[0]), "max_ms": float(kept[-1]),
            "std_ms": float(np.std(kept)), "runs": len(a), "kept": len(kept)}


def timed_steps(run, steps, dom_bit=None, timer=None):
    """Time exactly `steps` steps, each between its own HIP events on the current
    stream (no host synchronisation inside the timed region); the dominant
    stage is timed at the same time by the library's stage timers."""
    import torch
    stream = torch.cuda.current_stream()
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    ms = (C.c_double * 7)()
    cnt = (C.c_int * 7)()
    if dom_bit is not None:
        timer.lib.hyres_profile_enable(timer.h, 1 << dom_bit)
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    evs[0].record(stream)
    for i in range(steps):
        run(i)
        evs[i + 1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    dom_ms = None
    if dom_bit is not None:
        timer._lib.check(timer.lib.hyres_profile_read(timer.h, ms, cnt), "profile read")
        timer.lib.hyres_profile_enable(timer.h, 0)
        dom_ms = ms[dom_bit] / max(cnt[dom_bit], 1)
    per = [evs[i].elapsed_time(evs[i + 1]) for i in range(steps)]
    total = evs[0].elapsed_time(evs[steps])
    return {"ms_per_step": total / steps, "olympic": olympic(per), "wall_s": wall, "dom_ms": dom_ms}


def x_errors(X, ref):
    X = np.asarray(X, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    d = X - ref
    return {"X_rel": float(np.linalg.norm(d) / np.linalg.norm(ref)),
            "X_max_elem_rel": float(np.abs(d).max() / np.abs(ref).max())}


def cpu_info():
    model = platform.processor() or "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return model


def cpu_cores():
    try:
        from threadpoolctl import threadpool_info
        return max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:  # pragma: no cover
        return len(os.sched_getaffinity(0))


def time_oracle(fn, min_runs=3, max_runs=15, budget_s=20.0):
    """Runs the oracle at least `min_runs` times (more while the budget lasts,
    at most `max_runs`); returns (Olympic mean seconds, runs, last result)."""
    ts, out = [], None
    while len(ts) < max_runs:
        t0 = time.perf_counter()
        out = fn()
        ts.append(time.perf_counter() - t0)
        if len(ts) >= min_runs and sum(ts) + ts[-1] > budget_s:
            break
    o = olympic(ts)
    return o["mean_ms"], len(ts), out      # seconds (olympic() is unit-agnostic)


def rate_entry(voxels, t, bytes_):
    o = t["olympic"]["mean_ms"]
    return {"voxels_per_s": voxels / (t["ms_per_step"] * 1e-3), "ms_per_step": t["ms_per_step"],
            "olympic": t["olympic"], "wall_s": t["wall_s"],
            "algorithmic_bytes_per_step": bytes_, "hbm_gbs": bytes_ / (o * 1e-3) / 1e9,
            "hbm_frac": bytes_ / (o * 1e-3) / 1e9 / HBM_PEAK_GBS}


# ------------------------------------------------------------ headline (c2)
def measure_single(api, timer, Ys, dims, precision, steps, warmup, workload):
    import torch
    H, W, p, r, L = dims
    dn = api.Denoiser(H, W, p, r, L, dtype=torch.float32, precision=precision, device=Ys[0].device)
    run = lambda i: dn.run(Ys[i % len(Ys)])       # noqa: E731
    for i in range(max(warmup, 1)):
        run(i)
    torch.cuda.synchronize()
    stage_ms = timer.stages(run)
    work = stage_work([dims], precision)
    dom = max(stage_ms, key=lambda k: stage_ms[k])
    t = timed_steps(run, steps, STAGES.index(dom), timer)
    rl = {k: roofline_of(k, work, stage_ms[k], None) for k in stage_ms}
    e = rate_entry(float(H * W * p), t, solve_bytes([dims]))
    e.update(stages_ms=stage_ms, stage_rooflines=rl,
             roofline=roofline_of(dom, work, t["dom_ms"], load_traffic(workload + "/" + precision, dom)))
    return dn, e


def run_single(args, api, timer, synth):
    import torch
    cfg = synth.CONFIG_SHAPES[2]
    dims = (cfg["H"], cfg["W"], cfg["p"], cfg["r"], cfg["levels"])
    H, W, p, r, L = dims
    t0 = time.time()
    cube = synth.config_cube(2, keep_clean=False)
    log("generated %dx%dx%d cube in %.1f s" % (H, W, p, time.time() - t0))
    Y = torch.tensor(cube.Y, device="cuda")
    Ys = [Y, Y.clone()]          # two resident copies, alternated step by step
    precs = ["native", "mixed"] if args.precision == "both" else [args.precision]
    res, dns = {}, {}
    for prec in precs:
        dns[prec], res[prec] = measure_single(api, timer, Ys, dims, prec, args.steps, args.warmup, "single")
        log("%s %.3f ms/solve (olympic %.3f)" % (prec, res[prec]["ms_per_step"], res[prec]["olympic"]["mean_ms"]))
    cpu = None
    if not args.no_parity or not args.no_cpu_baseline:
        from oracle import hyres_oracle as O
        Y64 = cube.Y.astype(np.float64)
        cpu_s, runs, ref = time_oracle(lambda: O.hyres(Y64, r, L), min_runs=3,
                                       max_runs=1 if args.no_cpu_baseline else 15)
        cpu = (cpu_s, "Olympic mean of %d oracle solves of the same %dx%dx%d cube (FP64 numpy), %.2f s each"
               % (runs, H, W, p, cpu_s))
        for prec, m in res.items():
            dn = dns[prec]
            X = dn.run(Y).double().cpu().numpy()
            V = dn.V.T.cpu().numpy()
            cosines = np.linalg.svd(V.T @ ref["V"], compute_uv=False)
            err = x_errors(X, ref["X"])
            err.update({
                "sigma_max_rel": float(np.max(np.abs(dn.sigma.cpu().numpy() / ref["sigma"] - 1))),
                "evals_top_r_max_rel": float(np.max(np.abs(dn.evals.cpu().numpy()[:r] / ref["evals"][:r] - 1))),
                "subspace_max_angle_rad": float(np.arccos(np.clip(cosines.min(), -1.0, 1.0))),
                "V_max_abs_diff": float(np.max(np.abs(V - ref["V"]))),
                "lambda_max_rel_diff": float(np.max(np.abs(dn.lam.cpu().numpy() - ref["lam"]) / ref["lam"])),
                "gap_ratio": float(dn.gap.cpu()[0]),
            })
            m["errors_vs_fp64_oracle"] = err
    for prec in res:
        res[prec]["device_status"] = int(dns[prec].status.cpu()[0])
    workload = ("HyRes solve of a %dx%dx%d FP32 cube (Houston-2013 shape), rank %d, %d db2 levels, "
                "per-band SNR 5-20 dB, linear-mixing synthetic; two resident copies alternated" % dims)
    return res, float(H * W * p), workload, cpu


# ------------------------------------------------------- other workloads
def run_small_fp64(args, api, synth):
    """64 x 64 x 32 FP64 cube, rank 4, 3 levels (the oracle finishes it in milliseconds)."""
    import torch
    from oracle import hyres_oracle as O
    cube = synth.config_cube(1, keep_clean=False)
    H, W, p = cube.Y.shape
    r, L = 4, 3
    Y = torch.tensor(cube.Y, device="cuda")
    Ys = [Y, Y.clone()]
    dn = api.Denoiser(H, W, p, r, L, dtype=torch.float64, device=Y.device)
    run = lambda i: dn.run(Ys[i % 2])       # noqa: E731
    for i in range(max(args.warmup, 1)):
        run(i)
    t = timed_steps(run, args.steps)
    e = rate_entry(float(H * W * p), t, solve_bytes([(H, W, p, r, L)], elem=8))
    cpu_s, runs, ref = time_oracle(lambda: O.hyres(cube.Y, r, L), min_runs=15, max_runs=15)
    e["errors_vs_fp64_oracle"] = x_errors(dn.run(Y).cpu().numpy(), ref["X"])
    e["oracle_s"] = cpu_s
    e["oracle_runs"] = runs
    e["device_status"] = int(dn.status.cpu()[0])
    e["workload"] = "64x64x32 FP64 cube, rank 4, 3 levels, 10 dB, native FP64"
    return e


def run_grad(args, api, synth):
    """Forward + backward of the 256 x 256 x 191 FP32 cube (rank 6, 4 levels) at
    fixed thresholds; the gradient is compared with torch autograd through the
    FP64 oracle forward on the CPU."""
    import torch
    from oracle import hyres_oracle as O
    from oracle import grad as OG
    cube = synth.config_cube(4, keep_clean=False)
    Y = cube.Y
    H, W, p = Y.shape
    r, L = 6, 4
    Yt = torch.tensor(Y, device="cuda")
    ref = O.hyres(Y.astype(np.float64), r, L)
    # thresholds away from every kink: near each SURE threshold, the middle of
    # the widest gap between the 32 nearest coefficient magnitudes
    lam_np = np.empty(r)
    for k in range(r):
        a = np.sort(np.abs(ref["B"][k]))
        i0 = int(np.searchsorted(a, ref["lam"][k]))
        w = a[max(0, i0 - 16):i0 + 16]
        g = int(np.argmax(np.diff(w)))
        lam_np[k] = 0.5 * (w[g] + w[g + 1])
    lam = torch.tensor(lam_np, device="cuda")
    R = np.random.default_rng(2).standard_normal(Y.shape).astype(np.float32)
    dX = torch.tensor(R, device="cuda")
    dn = api.Denoiser(H, W, p, r, L, dtype=torch.float32, device=Yt.device)
    Ys = [Yt, Yt.clone()]
    out = {}

    def step(i):
        Yi = Ys[i % 2]
        dn.run(Yi, None, lam)
        out["g"] = api.denoise_backward(dn, Yi, dX)

    for i in range(max(args.warmup, 1)):
        step(i)
    t = timed_steps(step, args.steps)
    fwd = timed_steps(lambda i: dn.run(Ys[i % 2], None, lam), args.steps)
    nbytes = 2.0 * solve_bytes([(H, W, p, r, L)])      # backward: the forward's count (dX, Y, dY; images, coefficients)
    e = rate_entry(float(H * W * p), t, nbytes)
    e["forward_ms_per_step"] = fwd["ms_per_step"]
    e["backward_over_forward"] = (t["ms_per_step"] - fwd["ms_per_step"]) / fwd["ms_per_step"]
    step(0)
    torch.cuda.synchronize()
    dY, dlam, st = out["g"]
    Yg = torch.tensor(Y, dtype=torch.float64, requires_grad=True)
    lg = torch.tensor(lam_np, dtype=torch.float64, requires_grad=True)
    Xo = OG.hyres_forward(Yg, lg, r, L, sign_ref=torch.tensor(dn.V.T.cpu().numpy(), dtype=torch.float64))
    (Xo * torch.tensor(R, dtype=torch.float64)).sum().backward()
    gY, gl = Yg.grad.numpy(), lg.grad.numpy()
    e["errors_vs_fp64_oracle_gradient"] = {
        "dY_rel": float(np.linalg.norm(dY.double().cpu().numpy() - gY) / np.linalg.norm(gY)),
        "dlambda_rel": float(np.linalg.norm(dlam.cpu().numpy() - gl) / np.linalg.norm(gl))}
    e["device_status"] = int(st.cpu()[0])
    e["workload"] = ("forward + backward (vector-Jacobian product wrt the cube and the thresholds) of a "
                     "256x256x191 FP32 cube, rank 6, 4 levels, thresholds held fixed")
    return e


def run_batch(args, api, synth, precs):
    """64 uneven cubes, one HIP graph replay per step, transform tiles tuned first."""
    import torch
    from oracle import hyres_oracle as O
    t0 = time.time()
    cubes = synth.config3_cubes()
    log("generated %d cubes in %.1f s" % (len(cubes), time.time() - t0))
    Yt = [torch.tensor(c.Y, device="cuda") for c in cubes]
    shapes = [(c.Y.shape[0], c.Y.shape[1], c.Y.shape[2], c.rank, c.levels) for c in cubes]
    total = float(sum(c.Y.size for c in cubes))
    nbytes = solve_bytes(shapes)
    # the oracle on the smallest cube of each band-count class
    pick = {}
    for i, c in enumerate(cubes):
        q = c.Y.shape[2]
        if q not in pick or c.Y.size < cubes[pick[q]].Y.size:
            pick[q] = i
    order = sorted(pick.values())
    res = {}
    refs = None
    for prec in precs:
        b = api.Batch(Yt, [c.rank for c in cubes], [c.levels for c in cubes], precision=prec)
        b.run()
        b.autotune(os.path.join(ROOT, "gpurun_out", "dwt_tiles.json") if args.tune_cache is None
                   else args.tune_cache)
        for _ in range(max(args.warmup, 1)):
            b.launch_graph()
        t = timed_steps(lambda i: b.launch_graph(), args.steps)
        e = rate_entry(total, t, nbytes)
        e["device_status"] = max(int(b.info(i)["status"].cpu()[0]) for i in range(len(cubes)))
        if refs is None:
            c0 = time.perf_counter()
            refs = {i: O.hyres(cubes[i].Y.astype(np.float64), cubes[i].rank, cubes[i].levels) for i in order}
            vox = sum(cubes[i].Y.size for i in order)
            cpu = (time.perf_counter() - c0) * total / vox
        errs = [x_errors(b.X[i].double().cpu().numpy(), refs[i]["X"]) for i in order]
        e["errors_vs_fp64_oracle"] = {"cubes": order,
                                      "X_rel_max": max(x["X_rel"] for x in errs),
                                      "X_max_elem_rel_max": max(x["X_max_elem_rel"] for x in errs)}
        res[prec] = e
        log("batch %s %.3f ms/step (graph)" % (prec, t["ms_per_step"]))
        del b
    vox = sum(cubes[i].Y.size for i in order)
    return {"workload": ("64 uneven FP32 cubes (H, W in [128, 512], p in {103, 128, 191, 224}, rank 4-12, "
                         "4 db2 levels, 10 dB), %.3f G voxels, one HIP graph replay per step" % (total / 1e9)),
            "precisions": res,
            "oracle_estimate_s": cpu,
            "oracle_sample": "one oracle solve of the smallest cube of each band count (%d voxels), "
                             "scaled by voxels to the batch" % vox}


def run_tiled(args, api, synth, precs):
    """2048 x 2048 x 224 sliding window (25 tiles of 512^2, 32 px overlap)."""
    import torch
    from oracle import hyres_oracle as O
    t0 = time.time()
    cube = synth.config_cube(5, keep_clean=False)
    Yh = cube.Y
    del cube
    H, W, p = Yh.shape
    r, L, tile, ov = 10, 4, 512, 32
    log("generated %dx%dx%d cube in %.1f s" % (H, W, p, time.time() - t0))
    Y = torch.tensor(Yh, device="cuda")
    X = torch.empty_like(Y)
    sy, sx = api.tile_grid(H, tile, ov), api.tile_grid(W, tile, ov)
    shapes = [(tile, tile, p, r, L)] * (len(sy) * len(sx))
    nbytes = solve_bytes(shapes, blended_output=(H, W, p))
    # a window on the corner where tiles (0,0), (0,1), (1,0) and (1,1) overlap
    y0, y1, x0, x1 = 470, 522, 470, 522
    wy = [O.tile_weights_1d(s, tile, H, ov) for s in sy[:2]]
    wx = [O.tile_weights_1d(s, tile, W, ov) for s in sx[:2]]
    res = {}
    cpu = None
    for prec in precs:
        run = lambda i: api.denoise_tiled(Y, r, L, tile=tile, overlap=ov, precision=prec, X=X)   # noqa: E731
        for i in range(max(args.warmup, 1)):
            _, info = run(i)
        t = timed_steps(run, args.steps)
        e = rate_entry(float(H * W * p), t, nbytes)
        e["device_status"] = int(info["status"].cpu()[0])
        lam = info["lam"].cpu().numpy()
        acc = np.zeros((y1 - y0, x1 - x0, p))
        ws = np.zeros((y1 - y0, x1 - x0))
        t_or = time.perf_counter()
        for iy in range(2):
            a, b = max(y0, sy[iy]), min(y1, sy[iy] + tile)
            for ix in range(2):
                c0, c1 = max(x0, sx[ix]), min(x1, sx[ix] + tile)
                sub = Yh[sy[iy]:sy[iy] + tile, sx[ix]:sx[ix] + tile].astype(np.float64)
                Xt = O.hyres(sub, r, L, lam=lam[iy * len(sx) + ix])["X"]
                w2 = wy[iy][a - sy[iy]:b - sy[iy], None] * wx[ix][None, c0 - sx[ix]:c1 - sx[ix]]
                acc[a - y0:b - y0, c0 - x0:c1 - x0] += w2[:, :, None] * Xt[a - sy[iy]:b - sy[iy], c0 - sx[ix]:c1 - sx[ix]]
                ws[a - y0:b - y0, c0 - x0:c1 - x0] += w2
        if cpu is None:
            cpu = (time.perf_counter() - t_or) / 4 * len(shapes)
        e["errors_vs_fp64_oracle"] = dict(window=[y0, y1, x0, x1], thresholds="device's",
                                          **x_errors(X[y0:y1, x0:x1].double().cpu().numpy(), acc / ws[:, :, None]))
        res[prec] = e
        log("tiled %s %.3f ms/step" % (prec, t["ms_per_step"]))
    return {"workload": ("sliding-window HyRes of a %dx%dx%d FP32 cube, 25 tiles of 512x512 with 32 px overlap, "
                         "rank 10, 4 db2 levels, SNR 5-15 dB + dead columns + 1%% impulses" % (H, W, p)),
            "precisions": res,
            "oracle_estimate_s": cpu,
            "oracle_sample": "oracle solves of the 4 tiles around one seam corner (at the device's thresholds), "
                             "scaled to the 25 tiles (blend not timed)"}


# VALU lane-operations per band and sweep of the l1-l1 stage: forward
# elimination with the fused shrinkage and Bregman updates (t: 2, clip: 1,
# h - s + b1: 2, v: 2, clip: 1, u - b2 and its mask: 3, rhs: 3, pivot: 2) and
# the back substitution (1).
L1_OPS_PER_BAND_SWEEP = 17
# FP32 vector peak without packed math: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz
VALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12


def run_hyminor(args, api, synth):
    """HyMiNoR on the 349 x 1905 x 144 FP32 cube: HyRes (rank 8, 4 levels,
    native FP32), then the l1-l1 sparse-noise stage (lam 0.55, mu1 = mu2 = 1,
    50 sweeps) in place; the stage is also timed alone on the device's HyRes
    output and checked against the oracle on 2000 sampled pixels."""
    import torch
    from oracle import hyminor_oracle as HM
    cube = synth.config_cube(2, keep_clean=False)
    Yh = cube.Y
    H, W, p = Yh.shape
    r, L = 8, 4
    lam, mu1, mu2, K = 0.55, 1.0, 1.0, 50
    Y = torch.tensor(Yh, device="cuda")
    Ys = [Y, Y.clone()]
    dn = api.Denoiser(H, W, p, r, L, dtype=torch.float32, device=Y.device)
    l1 = api.L.L1Options(lam, mu1, mu2, K)
    run = lambda i: dn.run_hyminor(Ys[i % 2], l1)        # noqa: E731
    for i in range(max(args.warmup, 1)):
        run(i)
    t = timed_steps(run, args.steps)
    n = H * W
    e = rate_entry(float(n * p), t, solve_bytes([(H, W, p, r, L)]) + 2.0 * n * p * 4)
    # the stage alone on the device's HyRes output
    X1 = dn.run(Y).clone()
    Xs = torch.empty_like(X1)
    stage = lambda i: api.l1l1_spectral(X1, lam, mu1, mu2, K, X=Xs)     # noqa: E731
    for i in range(max(args.warmup, 1)):
        stage(i)
    ts = timed_steps(stage, args.steps)
    ms = ts["olympic"]["mean_ms"]
    ops = float(L1_OPS_PER_BAND_SWEEP) * p * K * n
    achieved = ops / (ms * 1e-3) / 1e12
    e["l1l1_ms"] = ms
    e["l1l1_olympic"] = ts["olympic"]
    e["roofline_l1l1"] = {"bound": "alu", "kernel": "l1l1", "achieved": achieved, "peak": VALU_PEAK_TOPS,
                          "unit": "Tops/s", "frac": achieved / VALU_PEAK_TOPS, "traffic": None, "kernel_ms": ms}
    rng = np.random.default_rng(4)
    idx = torch.tensor(rng.choice(n, 2000, replace=False), device="cuda")
    h = X1.reshape(n, p)[idx].cpu().numpy().astype(np.float64)
    got = Xs.reshape(n, p)[idx].cpu().numpy()
    t0 = time.perf_counter()
    ref = HM.l1l1_split_bregman(h, lam, mu1, mu2, K)
    cpu_stage = (time.perf_counter() - t0) * n / 2000
    e["errors_vs_fp64_oracle_stage"] = dict(pixels=2000, **x_errors(got, ref))
    e["oracle_stage_estimate_s"] = cpu_stage
    e["oracle_stage_sample"] = "oracle l1-l1 iteration on 2000 sampled pixels, scaled by pixels to the cube"
    e["device_status"] = int(dn.status.cpu()[0])
    e["workload"] = ("HyMiNoR of the 349x1905x144 FP32 cube: HyRes rank 8, 4 levels, native FP32, then the "
                     "per-pixel l1-l1 spectral stage, lam 0.55, mu1 = mu2 = 1, 50 sweeps")
    log("hyminor %.3f ms/step, l1l1 stage %.3f ms (%.2f of the VALU peak)" % (t["ms_per_step"], ms,
                                                                                achieved / VALU_PEAK_TOPS))
    return e


def run_wsrrr(args, api, synth):
    """WSRRR on the 349 x 1905 x 144 FP32 cube: HyRes (rank 8, 4 levels, native
    FP32), then 5 Procrustes / soft-threshold alternations at its thresholds;
    checked against the oracle at the device's noise and thresholds."""
    import torch
    from oracle import wsrrr_oracle as WO
    cube = synth.config_cube(2, keep_clean=False)
    Yh = cube.Y
    H, W, p = Yh.shape
    r, L, K = 8, 4, 5
    Y = torch.tensor(Yh, device="cuda")
    Ys = [Y, Y.clone()]
    run = lambda i: api.wsrrr(Ys[i % 2], r, L, K)        # noqa: E731
    for i in range(max(args.warmup, 1)):
        run(i)
    t = timed_steps(run, args.steps)
    n = H * W
    # the HyRes solve, then per alternation: Y and Zh read for Y^T Zh, the
    # projection (Y read, Z written), the two transforms, Zh written
    per_iter = 4.0 * (2 * n * p + 4 * n * r) + solve_bytes([(H, W, p, r, L)]) - 4.0 * (n * r + n * p)
    e = rate_entry(float(n * p), t, solve_bytes([(H, W, p, r, L)]) + K * per_iter)
    X, info = api.wsrrr(Y, r, L, K)
    t0 = time.perf_counter()
    ref = WO.wsrrr(Yh.astype(np.float64), r, L, K, sigma=info["sigma"].cpu().numpy(), lam=info["lam"].cpu().numpy())
    e["oracle_s"] = time.perf_counter() - t0
    e["oracle_sample"] = "one oracle run of the whole cube at the device's noise and thresholds"
    e["errors_vs_fp64_oracle"] = x_errors(X.cpu().numpy(), ref["X"])
    e["device_status"] = int(info["status"].cpu()[0])
    e["workload"] = ("WSRRR of the 349x1905x144 FP32 cube: HyRes rank 8, 4 levels, native FP32, then 5 "
                     "alternations of the Procrustes and soft-threshold steps")
    log("wsrrr %.3f ms/step" % t["ms_per_step"])
    return e


def run_forpdn(args, api, synth):
    """FORPDN on the 349 x 1905 x 144 FP32 cube, 4 levels, thresholds by SURE;
    checked against the oracle at the device's noise and thresholds on the
    whole cube (the oracle run is the CPU baseline of this workload)."""
    import torch
    from oracle import forpdn_oracle as FO
    cube = synth.config_cube(2, keep_clean=False)
    Yh = cube.Y
    H, W, p = Yh.shape
    L = 4
    Y = torch.tensor(Yh, device="cuda")
    Ys = [Y, Y.clone()]
    X = torch.empty_like(Y)
    run = lambda i: api.forpdn(Ys[i % 2], L, X=X)        # noqa: E731
    for i in range(max(args.warmup, 1)):
        run(i)
    t = timed_steps(run, args.steps)
    n = H * W
    # cube read twice (noise Gram, first analysis level), coefficients written
    # and read by the group Grams, the smoother and the synthesis (about one
    # cube each way), X written
    nbytes = 4.0 * n * p * 7
    e = rate_entry(float(n * p), t, nbytes)
    _, info = api.forpdn(Y, L, X=X)
    lam = info["lam"].cpu().numpy()
    sig = info["sigma"].cpu().numpy()
    t0 = time.perf_counter()
    ref = FO.forpdn(Yh.astype(np.float64), L, sigma=sig, lam=lam)
    e["oracle_s"] = time.perf_counter() - t0
    e["oracle_sample"] = "one oracle run of the whole cube at the device's noise and thresholds (no grid search)"
    e["errors_vs_fp64_oracle"] = x_errors(X.cpu().numpy(), ref["X"])
    e["lambda"] = [float(v) for v in lam]
    e["device_status"] = int(info["status"].cpu()[0])
    e["workload"] = ("FORPDN of the 349x1905x144 FP32 cube: regression noise, 4 db2 levels, first-order "
                     "spectral roughness smoother per wavelet group with SURE-chosen thresholds")
    log("forpdn %.3f ms/step" % t["ms_per_step"])
    return e


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=15)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--precision", default="both", choices=["native", "mixed", "both"])
    ap.add_argument("--workload", default="all", choices=["all", "single", "small", "grad", "batch", "tiled", "hyminor", "forpdn", "wsrrr"])
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
    precs = ["native", "mixed"] if args.precision == "both" else [args.precision]
    others = {}
    if args.workload in ("small", "grad", "batch", "tiled", "hyminor", "forpdn", "wsrrr"):
        # one secondary workload alone: its own line
        fn = {"small": lambda: run_small_fp64(args, api, synth), "grad": lambda: run_grad(args, api, synth),
              "batch": lambda: run_batch(args, api, synth, precs),
              "tiled": lambda: run_tiled(args, api, synth, precs),
              "hyminor": lambda: run_hyminor(args, api, synth),
              "forpdn": lambda: run_forpdn(args, api, synth),
              "wsrrr": lambda: run_wsrrr(args, api, synth)}[args.workload]
        e = fn()
        print(json.dumps({"metric": METRIC, "workload": args.workload, "n_gpus": 1, "steps": args.steps,
                          "warmup": args.warmup, "result": e}))
        return 0

    res, voxels, workload, cpu = run_single(args, api, timer, synth)
    if args.workload == "all":
        for name, fn in (("small_64x64x32_fp64", lambda: run_small_fp64(args, api, synth)),
                         ("grad_256x256x191_fwd_bwd", lambda: run_grad(args, api, synth)),
                         ("batch64", lambda: run_batch(args, api, synth, precs)),
                         ("tiled_2048x2048x224", lambda: run_tiled(args, api, synth, precs)),
                         ("hyminor_349x1905x144", lambda: run_hyminor(args, api, synth)),
                         ("forpdn_349x1905x144", lambda: run_forpdn(args, api, synth)),
                         ("wsrrr_349x1905x144", lambda: run_wsrrr(args, api, synth))):
            t0 = time.time()
            others[name] = fn()
            log("%s done in %.1f s" % (name, time.time() - t0))
            torch.cuda.empty_cache()
    head_prec = "mixed" if "mixed" in res else next(iter(res))
    head = res[head_prec]
    out = {
        "metric": METRIC,
        "value": voxels / (head["ms_per_step"] * 1e-3),
        "unit": "voxels/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16-split/f32" if head_prec == "mixed" else "f32",
        "data": "synthetic",
        "config": {"workload": workload, "precision": head_prec},
        "roofline": head["roofline"],
    }
    for prec, m in res.items():
        out["config"][prec] = m
    if others:
        out["config"]["workloads"] = others
    if cpu is not None and not args.no_cpu_baseline:
        cpu_s, sample = cpu
        out["cpu_baseline"] = {"value": voxels / cpu_s, "unit": "voxels/s", "cores": int(cpu_cores()),
                               "kind": "oracle", "sample": sample, "cpu_model": cpu_info()}
    print(json.dumps(out))
    return 0


if __name__ == "__main__":
    sys.exit(main())
