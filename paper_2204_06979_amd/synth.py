"""Seeded synthetic hyperspectral cubes (inputs only; no denoising arithmetic).

The paper evaluates HyRes on the Houston 2013 cube with added Gaussian noise
(Section 3) and mentions non-i.i.d., dead-line and impulse noise among the
simulators of the toolbox (Section 2, utility functions).  The dataset is not
available, so every workload here is a synthetic linear-mixing cube

    Y = A E^T + N,

with A (n x r) smooth abundance maps, E (p x r) smooth spectra and N Gaussian
noise at a prescribed per-band SNR, plus optional dead columns and impulses.
The same arrays feed the HIP path and the CPU oracle.

Recipe (fixed so that every run is reproducible):
  * RNG: numpy Generator(PCG64(seed)); draw order abundances, spectra, noise,
    corruption.
  * abundance maps: white N(0,1) fields filtered periodically in Fourier space
    by exp(-2 pi^2 s^2 |f|^2), s = l/sqrt(2) (correlation exp(-d^2/(2 l^2))),
    standardised per map, then softmax across the r maps at every pixel.
  * spectra: natural cubic spline through 6 knots at linspace(0, p-1, 6) with
    U[0,1] values, evaluated at 0..p-1, clipped to [0, 1].
  * noise: sigma_b = sqrt(mean_pixels(X_b^2) / 10^(SNR_b/10)), i.i.d. per voxel;
    each chunk of 65536 pixels draws from its own generator, spawned from a
    seed that the cube's generator draws after the spectra and SNRs.
  * dead columns: round(0.2 p) bands, round(0.05 W) columns each, set to 0.
  * impulses: 1% of voxels per band set to that band's min or max (p = 1/2),
    min/max taken just before impulses are applied; one uniform draw per
    voxel from a per-band generator (spawned like the noise seeds).
"""
from __future__ import annotations

import dataclasses
import os
from concurrent.futures import ThreadPoolExecutor
from typing import List, Optional, Sequence

import numpy as np
from scipy.interpolate import CubicSpline

__all__ = [
    "Cube", "abundances", "spectra", "mixing_cube", "config_cube",
    "config3_cubes", "tile_starts", "CONFIG_SHAPES",
]


@dataclasses.dataclass
class Cube:
    """A noisy cube with its ground truth.  Arrays are H x W x p."""
    Y: np.ndarray                 # noisy cube (dtype as requested)
    X: Optional[np.ndarray]       # clean cube (float64) or None when not kept
    sigma_true: np.ndarray        # per-band noise std actually used (float64, p)
    rank: int
    levels: int
    seed: int

    @property
    def shape(self):
        return self.Y.shape


def _rng(seed) -> np.random.Generator:
    if isinstance(seed, np.random.SeedSequence):
        return np.random.Generator(np.random.PCG64(seed))
    return np.random.Generator(np.random.PCG64(int(seed)))


def abundances(rng: np.random.Generator, H: int, W: int, r: int,
               length_scale: float = 8.0) -> np.ndarray:
    """r smooth maps (Gaussian random fields), softmax-normalised per pixel.

    Returns an (H*W) x r float64 array, row index = y*W + x.
    """
    s = length_scale / np.sqrt(2.0)
    fy = np.fft.fftfreq(H)[:, None]
    fx = np.fft.rfftfreq(W)[None, :]
    transfer = np.exp(-2.0 * np.pi ** 2 * s ** 2 * (fx ** 2 + fy ** 2))
    maps = np.empty((r, H, W))
    for i in range(r):
        white = rng.standard_normal((H, W))
        f = np.fft.irfft2(np.fft.rfft2(white) * transfer, s=(H, W))
        f = (f - f.mean()) / f.std()
        maps[i] = f
    maps -= maps.max(axis=0, keepdims=True)
    e = np.exp(maps)
    e /= e.sum(axis=0, keepdims=True)
    return e.reshape(r, H * W).T.copy()


def spectra(rng: np.random.Generator, p: int, r: int, knots: int = 6) -> np.ndarray:
    """r smooth spectra in [0,1]; returns p x r float64."""
    xk = np.linspace(0.0, p - 1.0, knots)
    xb = np.arange(p, dtype=np.float64)
    E = np.empty((p, r))
    for i in range(r):
        yk = rng.uniform(0.0, 1.0, size=knots)
        E[:, i] = np.clip(CubicSpline(xk, yk, bc_type="natural")(xb), 0.0, 1.0)
    return E


def _pool(workers: int, jobs: int) -> int:
    return max(1, min(workers if workers else (os.cpu_count() or 1), 16, jobs))


def mixing_cube(seed, H: int, W: int, p: int, r: int, snr_db, levels: int,
                dtype=np.float32, keep_clean: bool = True,
                dead_columns: bool = False, impulses: bool = False,
                row_chunk: int = 1 << 16, workers: int = 0) -> Cube:
    """Y = A E^T + N (+ optional dead columns and impulses), H x W x p.

    ``snr_db`` is a scalar (same SNR for every band) or a pair (lo, hi) for a
    per-band SNR drawn uniformly in [lo, hi] dB.  The noise of each chunk of
    ``row_chunk`` pixels and the impulses of each band come from their own
    generators, spawned from one seed drawn by the cube's generator, so the
    work runs on ``workers`` threads (0: all cores) with values that do not
    depend on the thread count, and multi-GB cubes fit in host memory.
    """
    rng = _rng(seed)
    n = H * W
    A = abundances(rng, H, W, r)
    E = spectra(rng, p, r)
    if np.ndim(snr_db) == 0:
        snr = np.full(p, float(snr_db))
    else:
        lo, hi = snr_db
        snr = rng.uniform(lo, hi, size=p)
    noise_seed = np.random.SeedSequence(int(rng.integers(0, 2 ** 63 - 1)))
    starts = list(range(0, n, row_chunk))
    nw = _pool(workers, len(starts))

    # mean-square signal power per band
    def power_of(s0):
        Xc = A[s0:s0 + row_chunk] @ E.T
        return np.einsum("ij,ij->j", Xc, Xc)

    with ThreadPoolExecutor(nw) as ex:
        power = np.sum(list(ex.map(power_of, starts)), axis=0) / n
    sigma = np.sqrt(power / 10.0 ** (snr / 10.0))
    Y = np.empty((n, p), dtype=dtype)
    X = np.empty((n, p), dtype=np.float64) if keep_clean else None

    def fill(job):
        s0, ss = job
        Xc = A[s0:s0 + row_chunk] @ E.T
        Nc = _rng(ss).standard_normal(Xc.shape) * sigma[None, :]
        Y[s0:s0 + row_chunk] = Xc + Nc
        if keep_clean:
            X[s0:s0 + row_chunk] = Xc

    with ThreadPoolExecutor(nw) as ex:
        list(ex.map(fill, zip(starts, noise_seed.spawn(len(starts)))))
    Y3 = Y.reshape(H, W, p)
    if dead_columns:
        nb = int(round(0.2 * p))
        nc = int(round(0.05 * W))
        bands = rng.choice(p, size=nb, replace=False)
        for b in bands:
            cols = rng.choice(W, size=nc, replace=False)
            Y3[:, cols, b] = 0
    if impulses:
        imp_seed = np.random.SeedSequence(int(rng.integers(0, 2 ** 63 - 1)))

        # one uniform draw per voxel: below 0.005 the band maximum, in [0.005, 0.01) the minimum
        def corrupt(job):
            b, ss = job
            band = Y3[:, :, b]
            lo_v, hi_v = band.min(), band.max()
            u = _rng(ss).random((H, W))
            band[u < 0.005] = hi_v
            band[(u >= 0.005) & (u < 0.01)] = lo_v

        with ThreadPoolExecutor(_pool(workers, p)) as ex:
            list(ex.map(corrupt, zip(range(p), imp_seed.spawn(p))))
    return Cube(Y=Y3, X=None if X is None else X.reshape(H, W, p),
                sigma_true=sigma, rank=r, levels=levels,
                seed=seed if not isinstance(seed, np.random.SeedSequence) else -1)


# Shapes of the five workloads: (H, W, p, r, levels, snr, dtype, seed)
CONFIG_SHAPES = {
    1: dict(H=64, W=64, p=32, r=4, levels=3, snr_db=10.0, dtype=np.float64, seed=1),
    2: dict(H=349, W=1905, p=144, r=8, levels=4, snr_db=(5.0, 20.0), dtype=np.float32, seed=2),
    4: dict(H=256, W=256, p=191, r=6, levels=4, snr_db=10.0, dtype=np.float32, seed=4),
    5: dict(H=2048, W=2048, p=224, r=10, levels=4, snr_db=(5.0, 15.0), dtype=np.float32, seed=5,
            dead_columns=True, impulses=True),
}


def config_cube(cfg: int, keep_clean: bool = True, **over) -> Cube:
    """The single-cube workloads 1, 2, 4 and 5 (config 3 is a list)."""
    kw = dict(CONFIG_SHAPES[cfg])
    kw.update(over)
    seed = kw.pop("seed")
    return mixing_cube(seed, keep_clean=keep_clean, **kw)


def config3_cubes(count: int = 64, keep_clean: bool = False,
                  hw_range=(128, 512), bands=(103, 128, 191, 224),
                  ranks=(4, 12), levels: int = 4, workers: int = 0) -> List[Cube]:
    """Workload 3: independent cubes of uneven size, one seed stream each."""
    specs = []
    for ss in np.random.SeedSequence(3).spawn(count):
        rng = _rng(ss)
        H = int(rng.integers(hw_range[0], hw_range[1] + 1))
        W = int(rng.integers(hw_range[0], hw_range[1] + 1))
        p = int(rng.choice(np.asarray(bands)))
        r = int(rng.integers(ranks[0], ranks[1] + 1))
        sub = rng.integers(0, 2 ** 63 - 1)
        specs.append((int(sub), H, W, p, r))

    def one(spec):
        sub, H, W, p, r = spec
        return mixing_cube(sub, H, W, p, r, 10.0, levels, dtype=np.float32, keep_clean=keep_clean, workers=1)

    # every cube has its own seed, so the worker count does not change the values
    workers = max(1, min(workers if workers else (os.cpu_count() or 1), 16, count))
    if workers == 1:
        return [one(s) for s in specs]
    with ThreadPoolExecutor(workers) as ex:
        return list(ex.map(one, specs))


def tile_starts(size: int, tile: int, overlap: int) -> List[int]:
    """Start offsets of sliding-window tiles along one axis (last one clamped)."""
    if tile >= size:
        return [0]
    step = tile - overlap
    starts = []
    k = 0
    while True:
        s = min(k * step, size - tile)
        starts.append(s)
        if s + tile >= size:
            break
        k += 1
    return starts
