"""Seeded synthetic inputs: determinism and the stated workload properties."""
import math

import numpy as np

from paper_2503_02412_amd import inputs as I


def test_generators_are_deterministic():
    assert np.array_equal(I.config1_map(1), I.config1_map(1))
    assert np.array_equal(I.config2_map(2), I.config2_map(2), equal_nan=True)
    assert not np.array_equal(I.config1_map(1), I.config1_map(2))


def test_config1_map_properties():
    h = I.config1_map(1)
    assert h.shape == (64, 64) and h.dtype == np.float32
    assert np.all(np.isfinite(h))
    assert np.abs(h).max() < 8 * 0.3 + 0.2


def test_config2_map_properties():
    h = I.config2_map(2)
    assert h.shape == (200, 200) and h.dtype == np.float32
    frac = np.isnan(h).mean()
    assert 0.05 <= frac < 0.06
    # Steps aside, the noise surface was rescaled to a 30 degree maximum slope.
    rng = np.random.Generator(np.random.PCG64(2))
    base = I.value_noise(200, 200, 0.1, rng)
    base *= math.tan(math.radians(30)) / I._max_slope(base, 0.1)
    assert abs(I._max_slope(base, 0.1) - math.tan(math.radians(30))) < 1e-9


def test_config5_hole_fraction():
    h = I.config5_map(5)
    assert h.shape == (800, 800)
    assert 0.15 <= np.isnan(h).mean() < 0.16


def test_trajectory_steps():
    t = I.trajectory(3)
    assert t.shape == (101, 2)
    steps = np.linalg.norm(np.diff(t, axis=0), axis=1)
    assert np.allclose(steps, 0.5)


def test_world_window_extraction():
    w, traj = I.rolling_world(I.CONFIG3)
    win = w.window(w.gx0 + 3, w.gy0 + 5, 10, 7)
    assert np.array_equal(win, w.heights[5:12, 3:13], equal_nan=True)
    out = w.window(w.gx0 - 4, w.gy0, 10, 2)
    assert np.all(np.isnan(out[:, :4]))


def test_pool2_means_known_cells_per_parity():
    from paper_2503_02412_amd.surrogate import pool2
    a = np.arange(16, dtype=np.float32).reshape(1, 4, 4)
    a[0, 0, 0] = np.nan
    a[0, 2, 3] = np.inf                       # not a known height
    assert np.allclose(pool2(a, 0, 0)[0], [[10 / 3, 4.5], [10.5, (10 + 14 + 15) / 3]])
    assert np.allclose(pool2(a, 1, 1)[0], [[7.5, 7.0], [13.5, 15.0]])
    assert np.allclose(pool2(a, 0, 1)[0], [[3.5, 5.0], [11.5, 15.0]])
    b = np.full((1, 2, 2), np.nan, np.float32)
    assert np.isnan(pool2(b, 0, 0)).all() and pool2(b, 1, 1).shape == (1, 1, 1)
