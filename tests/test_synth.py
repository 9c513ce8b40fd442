"""The seeded workload generator: determinism and the stated recipe."""
import numpy as np

from paper_2204_06979_amd import synth


def test_generator_is_deterministic_and_matches_recipe():
    a = synth.config_cube(1)
    b = synth.config_cube(1)
    assert a.Y.dtype == np.float64 and a.Y.shape == (64, 64, 32)
    np.testing.assert_array_equal(a.Y, b.Y)
    X = a.X.reshape(-1, 32)
    N = (a.Y - a.X).reshape(-1, 32)
    snr = 10 * np.log10((X ** 2).mean(0) / a.sigma_true ** 2)
    np.testing.assert_allclose(snr, 10.0, atol=1e-9)
    # empirical noise std close to the prescribed one
    assert np.abs(N.std(0) / a.sigma_true - 1).max() < 0.1
    assert X.min() >= 0 and X.max() <= 1


def test_abundances_sum_to_one_and_spectra_in_unit_interval():
    rng = np.random.default_rng(0)
    A = synth.abundances(rng, 40, 30, 5)
    np.testing.assert_allclose(A.sum(1), 1.0, atol=1e-12)
    E = synth.spectra(rng, 50, 5)
    assert E.min() >= 0 and E.max() <= 1


def test_corruptions_for_the_sliding_window_recipe():
    c = synth.mixing_cube(5, 64, 80, 20, 3, (5, 15), 2, keep_clean=False,
                          dead_columns=True)
    Y = c.Y
    dead = [(b, x) for b in range(20) for x in range(80) if np.all(Y[:, x, b] == 0)]
    assert len({b for b, _ in dead}) == 4                   # round(0.2 p)
    assert len(dead) == 4 * 4                               # round(0.05 W) columns per band
    c2 = synth.mixing_cube(5, 64, 80, 20, 3, (5, 15), 2, keep_clean=False,
                           dead_columns=True, impulses=True)
    frac = []
    for b in range(20):
        band = c2.Y[:, :, b]
        frac.append(np.mean((band == band.min()) | (band == band.max())))
    assert 0.005 < np.mean(frac) < 0.02                     # about 1% impulses


def test_batched_workload_shapes():
    cubes = synth.config3_cubes(count=4, hw_range=(16, 40), levels=2)
    for c in cubes:
        H, W, p = c.Y.shape
        assert 16 <= H <= 40 and 16 <= W <= 40 and p in (103, 128, 191, 224)
        assert 4 <= c.rank <= 12
