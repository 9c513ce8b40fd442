"""Pins of the HyMiNoR sparse-noise oracle against facts that do not come from
the oracle itself: the optimum of the l1-l1 problem as a linear program,
closed-form minimisers (an isolated spectral spike is removed exactly when
lam > 1/2 and kept when lam < 1/2; a flat spectrum is a fixed point of every
sweep), the exact scaling law of the iteration, and the effect on a cube with
dead columns."""
import numpy as np
import pytest
from scipy import optimize

from oracle import hyminor_oracle as HM
from oracle import hyres_oracle as O
from paper_2204_06979_amd import synth


def _lp_optimum(h, lam):
    """min ||h - x||_1 + lam ||x_{i+1} - x_i||_1 as a linear program in (x, t, w)."""
    p = h.size
    Dm = np.diff(np.eye(p), axis=0)                 # rows e_{i+1} - e_i
    I, Z = np.eye(p), np.zeros((p - 1, p))
    c = np.concatenate([np.zeros(p), np.ones(p), lam * np.ones(p - 1)])
    A = np.block([[-I, -I, np.zeros((p, p - 1))],
                  [I, -I, np.zeros((p, p - 1))],
                  [Dm, Z, -np.eye(p - 1)],
                  [-Dm, Z, -np.eye(p - 1)]])
    b = np.concatenate([-h, h, np.zeros(p - 1), np.zeros(p - 1)])
    bounds = [(None, None)] * p + [(0, None)] * (2 * p - 1)
    res = optimize.linprog(c, A_ub=A, b_ub=b, bounds=bounds, method="highs")
    assert res.status == 0
    return res.fun, res.x[:p]


@pytest.mark.parametrize("lam", [0.3, 0.8, 2.0])
def test_converged_iteration_reaches_the_linear_program_optimum(lam):
    rng = np.random.default_rng(11)
    p = 12
    hs = []
    for k in range(6):
        h = np.cumsum(rng.standard_normal(p)) * 0.2 + 1.0
        h[rng.integers(0, p, 2)] += rng.choice([-2.0, 3.0], 2)      # sparse spikes
        hs.append(h)
    Hc = np.stack(hs)
    x = HM.l1l1_split_bregman(Hc, lam, 1.0, 1.0, 6000)
    for k in range(len(hs)):
        opt, _ = _lp_optimum(hs[k], lam)
        got = HM.l1l1_objective(hs[k], x[k], lam)
        assert got - opt <= 1e-6 * max(1.0, opt), (k, got, opt)
        assert got >= opt - 1e-7


@pytest.mark.parametrize("lam,removed", [(0.8, True), (3.0, True), (0.3, False)])
def test_isolated_spike(lam, removed):
    # flat spectrum c plus a spike a at an interior band: removing it costs |a|
    # in the data term and saves 2 lam |a| of roughness
    p, c, a = 9, 0.7, 2.5
    h = np.full(p, c)
    h[4] += a
    x = HM.l1l1_split_bregman(h[None], lam, 1.0, 1.0, 5000)[0]
    want = np.full(p, c) if removed else h
    np.testing.assert_allclose(x, want, atol=1e-6)


@pytest.mark.parametrize("iters", [1, 2, 7])
def test_flat_spectrum_is_a_fixed_point(iters):
    h = np.full((3, 17), 0.25)
    x = HM.l1l1_split_bregman(h, 1.5, 0.7, 0.3, iters)
    np.testing.assert_allclose(x, h, rtol=0, atol=1e-15)


def test_zero_roughness_weight_returns_the_input():
    rng = np.random.default_rng(3)
    h = rng.standard_normal((4, 10))
    x = HM.l1l1_split_bregman(h, 0.0, 1.0, 1.0, 3000)
    np.testing.assert_allclose(x, h, atol=1e-7)


def test_scaling_law_of_the_iteration():
    # scaling the data by a and the penalties by 1/a scales every iterate by a
    rng = np.random.default_rng(5)
    h = rng.standard_normal((5, 14))
    a = 3.0
    x1 = HM.l1l1_split_bregman(h, 0.9, 0.6, 0.2, 9)
    xa = HM.l1l1_split_bregman(a * h, 0.9, 0.6 / a, 0.2 / a, 9)
    np.testing.assert_allclose(xa, a * x1, rtol=1e-12, atol=1e-13)
    # and the iterate is not the input (the pin has something to scale)
    assert np.abs(x1 - h).max() > 1e-2


def test_spectral_difference_rows():
    D = HM.spectral_difference(4)
    x = np.array([1.0, 4.0, 9.0, 16.0])
    np.testing.assert_array_equal(D @ x, [3.0, 5.0, 7.0])
    assert HM.spectral_difference(1).shape == (0, 1)


def test_rejects_bad_parameters():
    h = np.zeros((1, 4))
    for args in [(1.0, 0.0, 1.0, 3), (1.0, 1.0, -1.0, 3), (-1.0, 1.0, 1.0, 3), (1.0, 1.0, 1.0, 0)]:
        with pytest.raises(ValueError):
            HM.l1l1_split_bregman(h, *args)


def test_sparse_stage_removes_stripes_left_by_hyres():
    # dead columns: at a rank above the signal's, HyRes keeps them as
    # components of their own, so its output still carries one-band dips along
    # those columns; the l1-l1 stage removes them
    cube = synth.mixing_cube(21, 64, 64, 32, 3, 20.0, 3, dtype=np.float64, keep_clean=True,
                             dead_columns=True)
    out = HM.hyminor(cube.Y, 8, 3, 0.55, 1.0, 1.0, 50)
    e_hyres = np.linalg.norm(out["X_hyres"] - cube.X)
    e_hyminor = np.linalg.norm(out["X"] - cube.X)
    assert e_hyminor < 0.7 * e_hyres, (e_hyminor, e_hyres)
    np.testing.assert_allclose(out["X_hyres"], O.hyres(cube.Y, 8, 3)["X"], rtol=0, atol=0)
