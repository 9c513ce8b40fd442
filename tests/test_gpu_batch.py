"""Batched solves of uneven cubes (needs an MI355X).

A batch runs every cube through the same kernels as a single-cube call, only
with work tables that span all cubes, so each cube's output must be bitwise
equal to hyres_denoise on that cube alone; one cube per batch is also checked
against the FP64 oracle directly.  The transform tile shape does not change
any coefficient, so results before and after autotuning are bitwise equal too.
"""
import json
import sys

import numpy as np
import pytest

from oracle import hyres_oracle as O
from paper_2204_06979_amd import synth

import parity_metrics as PM
import sure_protocol as SP

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _api():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2204_06979_amd import api
    return api


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


# shapes chosen to span several band-tile classes (T = 1, 2, 3, 7, 8, 11, 12, 14), the
# small-solve register tilings, odd sizes and differing ranks and levels
SHAPES = [(97, 133, 40, 5, 3), (64, 200, 17, 1, 2), (150, 77, 103, 8, 3), (128, 128, 128, 6, 4),
          (45, 61, 191, 4, 2), (130, 90, 224, 12, 3), (33, 40, 2, 2, 2), (81, 81, 48, 3, 4),
          (70, 90, 170, 5, 3)]


def _cubes(dtype, shapes=SHAPES):
    out = []
    for k, (H, W, p, r, L) in enumerate(shapes):
        c = synth.mixing_cube(1000 + k, H, W, p, min(r, 6), 12.0, L, dtype=np.float64, keep_clean=False)
        Y = c.Y + 1e-3 * np.random.default_rng(k).standard_normal(c.Y.shape)
        out.append(Y.astype(dtype))
    return out


def _run_batch(api, Ys, prec, graph=False, lams=None):
    cubes = [torch.tensor(Y, device="cuda") for Y in Ys]
    b = api.Batch(cubes, [s[3] for s in SHAPES[:len(Ys)]], [s[4] for s in SHAPES[:len(Ys)]], precision=prec,
                  lams=lams)
    if graph:
        b.launch_graph()
    else:
        b.run()
    torch.cuda.synchronize()
    return b


@pytest.mark.parametrize("dtype,prec", [(np.float32, "native"), (np.float32, "mixed"), (np.float64, "native")])
def test_batch_equals_single_cube_runs(dtype, prec):
    api = _api()
    Ys = _cubes(dtype)
    say("batch", dtype.__name__, prec, len(Ys), "cubes")
    b = _run_batch(api, Ys, prec)
    for i, Y in enumerate(Ys):
        H, W, p, r, L = SHAPES[i]
        X1, info1 = api.denoise(torch.tensor(Y, device="cuda"), r, L, precision=prec)
        inf = b.info(i)
        assert int(inf["status"].cpu()[0]) & ~8 == 0, (i, int(inf["status"].cpu()[0]))
        assert torch.equal(b.X[i], X1), i
        assert torch.equal(inf["lam"], info1["lam"]), i
        assert torch.equal(inf["sigma"], info1["sigma"]), i
        assert torch.equal(inf["V"], info1["V"]), i
    # cubes straight against the oracle: 103 bands, and the widest (224 bands,
    # three-part native Gram and the largest small-solve tiling)
    tol = {np.float64: 1e-10, np.float32: 1e-5}[dtype] if prec == "native" else 1e-3
    for i in (2, 5):
        H, W, p, r, L = SHAPES[i]
        ref = O.hyres(Ys[i].astype(np.float64), r, L, lam=b.info(i)["lam"].cpu().numpy())
        e, emax = PM.assert_close(b.X[i].cpu().numpy(), ref["X"], tol, "cube %d" % i)
        say("  oracle cube", i, "p", p, "rel err", e, "max err / max", emax)


def test_batch_graph_replays_match_eager():
    api = _api()
    Ys = _cubes(np.float32)
    b = _run_batch(api, Ys, "mixed")
    eager = [x.clone() for x in b.X]
    lam = [b.info(i)["lam"].clone() for i in range(len(Ys))]
    for rep in range(3):
        for x in b.X:
            x.zero_()
        b.launch_graph()
        torch.cuda.synchronize()
        for i in range(len(Ys)):
            assert torch.equal(b.X[i], eager[i]), (rep, i)
            assert torch.equal(b.info(i)["lam"], lam[i]), (rep, i)
        # eager work between replays
        b.run()
        torch.cuda.synchronize()
        for i in range(len(Ys)):
            assert torch.equal(b.X[i], eager[i]), ("eager", rep, i)


def test_batch_with_given_thresholds_on_some_cubes():
    api = _api()
    Ys = _cubes(np.float64)[:4]
    lams = [None, torch.tensor([0.5]), None, torch.linspace(0.2, 1.2, SHAPES[3][3], dtype=torch.float64)]
    b = _run_batch(api, Ys, "native", lams=lams)
    for i in range(4):
        H, W, p, r, L = SHAPES[i]
        lam_i = None if lams[i] is None else lams[i].numpy()
        ref = O.hyres(Ys[i], r, L, lam=lam_i if lam_i is not None else b.info(i)["lam"].cpu().numpy())
        if lam_i is None:
            # the SURE choice itself against the oracle's (a different candidate
            # only where its oracle risk ties the minimum to 1e-6 N)
            ref_sure = O.hyres(Ys[i], r, L)
            got = b.info(i)["lam"].cpu().numpy()
            for k in range(r):
                if got[k] != ref_sure["lam"][k]:
                    ok, gap, allowed = SP.accept(ref_sure["B"][k], got[k], ref_sure["lam"][k], ref_sure["sure"][k],
                                                 SP.EPS["float64"])
                    assert ok, (i, k, gap, allowed)
        else:
            np.testing.assert_array_equal(b.info(i)["lam"].cpu().numpy(), lam_i)
        PM.assert_close(b.X[i].cpu().numpy(), ref["X"], 1e-10, "cube %d" % i)


def test_autotune_cache_and_unchanged_results(tmp_path):
    api = _api()
    Ys = _cubes(np.float32)
    b = _run_batch(api, Ys, "mixed")
    before = [x.clone() for x in b.X]
    path = str(tmp_path / "tiles.json")
    b.autotune(path)
    data = json.load(open(path))
    assert data["format"] == "hyres-dwt-tiles-1"
    ents = data["entries"]
    assert len(ents) > 0
    for e in ents:
        assert (e["tx"], e["ty"]) in [(64, 4), (32, 8), (16, 16), (128, 2)]
    # every width class of the batch is tuned now
    for H, W, p, r, L in SHAPES:
        w = W
        for l in range(L):
            w = (w + 1) // 2
            for inv in (False, True):
                tx, ty, tuned = api.tile_choice(torch.float32, inv, w)
                assert tuned, (w, inv)
    b.run()
    torch.cuda.synchronize()
    for i in range(len(Ys)):
        assert torch.equal(b.X[i], before[i]), i
    # the graph captured after tuning gives the same result
    b.launch_graph()
    torch.cuda.synchronize()
    for i in range(len(Ys)):
        assert torch.equal(b.X[i], before[i]), i
    # a second tune reads the cache and keeps the file's choices
    b.autotune(path)
    assert json.load(open(path))["entries"] == ents


@pytest.mark.slow
def test_config3_batch_64_uneven_cubes():
    api = _api()
    cubes = synth.config3_cubes()
    say("config3", len(cubes), "cubes,", sum(c.Y.size for c in cubes) / 1e9, "G voxels")
    Yt = [torch.tensor(c.Y, device="cuda") for c in cubes]
    b = api.Batch(Yt, [c.rank for c in cubes], [c.levels for c in cubes], precision="mixed")
    b.launch_graph()
    torch.cuda.synchronize()
    bad = [i for i in range(len(cubes)) if int(b.info(i)["status"].cpu()[0]) & ~8]
    assert not bad, bad
    # every cube equals its single-cube solve
    for i, c in enumerate(cubes):
        X1, info1 = api.denoise(Yt[i], c.rank, c.levels, precision="mixed")
        assert torch.equal(b.X[i], X1), i
    # against the oracle (at the device's thresholds): the two smallest cubes,
    # and the smallest cube of each of the two widest band counts
    order = sorted(range(len(cubes)), key=lambda i: cubes[i].Y.size)
    pick = order[:2]
    for pb in (224, 191):
        pick += [next(i for i in order if cubes[i].Y.shape[2] == pb and i not in pick)]
    for i in pick:
        c = cubes[i]
        ref = O.hyres(c.Y.astype(np.float64), c.rank, c.levels, lam=b.info(i)["lam"].cpu().numpy())
        e, emax = PM.assert_close(b.X[i].cpu().numpy(), ref["X"], 1e-3, "cube %d" % i)
        say("  cube", i, c.Y.shape, "rank", c.rank, "rel err", e, "max err / max", emax)
