"""Pins of the FP64 SDF / trilinear-query reference (oracle/sdf.py) against
an independent exact EDT (scipy), closed forms and the interpolant's
defining properties."""
import math

import numpy as np
import pytest
from scipy import ndimage

from oracle import sdf as S


def scipy_sdf(obst, res, cap):
    """The same field from scipy's exact Euclidean distance transform."""
    d_obst = ndimage.distance_transform_edt(~obst) if obst.any() else np.full(obst.shape, np.inf)
    d_free = ndimage.distance_transform_edt(obst) if (~obst).any() else np.full(obst.shape, np.inf)
    return np.where(obst, -(np.minimum(d_free, cap) - 0.5), np.minimum(d_obst, cap) - 0.5) * res


@pytest.mark.parametrize("seed,shape,cap,frac", [(1, (23, 31), 40, 0.1), (2, (40, 17), 6, 0.3),
                                                 (3, (12, 12), 3, 0.02), (4, (30, 30), 100, 0.6)])
def test_sdf_matches_scipy_edt(seed, shape, cap, frac):
    rng = np.random.default_rng(seed)
    obst = rng.random(shape) < frac
    got = S.sdf_plane(obst, 0.05, cap)
    assert np.max(np.abs(got - scipy_sdf(obst, 0.05, cap))) < 1e-12


def test_single_obstacle_closed_form():
    H, W, res, cap = 21, 25, 0.1, 8
    obst = np.zeros((H, W), bool)
    obst[7, 11] = True
    got = S.sdf_plane(obst, res, cap)
    ys, xs = np.mgrid[0:H, 0:W]
    d = np.minimum(np.hypot(xs - 11, ys - 7), cap)
    want = (d - 0.5) * res
    want[7, 11] = -0.5 * res               # the nearest free cell is one cell away
    assert np.max(np.abs(got - want)) < 1e-12


def test_empty_and_full_planes_and_unknown_states():
    res, cap = 0.1, 5
    assert np.all(S.sdf_plane(np.zeros((6, 7), bool), res, cap) == (cap - 0.5) * res)
    assert np.all(S.sdf_plane(np.ones((6, 7), bool), res, cap) == -(cap - 0.5) * res)
    st = np.full((1, 4, 5), 1 | 16, np.uint8)          # valid, traversable
    st[0, 2, 2] = 0                                       # UNKNOWN
    st[0, 0, 4] = 1 | 4                                   # tilt obstacle
    a = S.sdf_planes(st, res, cap, unknown_is_obstacle=True)
    b = S.sdf_planes(st, res, cap, unknown_is_obstacle=False)
    assert a[0, 2, 2] < 0 and b[0, 2, 2] > 0 and a[0, 0, 4] < 0 and b[0, 0, 4] < 0


def test_surrogate_answers_count_as_obstacles_unless_traversable():
    """Surrogate states (bit 32) carry no curvature or tilt bit; those not
    traversable are obstacles, the traversable ones free.  Near-degenerate and
    traversable bits alone never make an obstacle."""
    st = np.full((1, 3, 4), 1 | 16, np.uint8)
    st[0, 0, 0] = 1 | 32                 # surrogate, not traversable -> obstacle
    st[0, 1, 1] = 1 | 16 | 32            # surrogate, traversable -> free
    st[0, 2, 2] = 1 | 8                  # plain, near-degenerate, risk > r_max -> free
    st[0, 2, 3] = 1 | 8 | 32             # surrogate (bit 8 ignored), not traversable
    m = S.obstacle_mask(st, unknown_is_obstacle=False)
    want = np.zeros((1, 3, 4), bool)
    want[0, 0, 0] = want[0, 2, 3] = True
    assert np.array_equal(m, want)


def grid_and_res():
    rng = np.random.default_rng(9)
    return rng.normal(size=(6, 9, 11)), 0.1


def test_query_reproduces_nodes():
    g, res = grid_and_res()
    K, H, W = g.shape
    poses, want = [], []
    for k in range(K):
        for j in (0, 4, H - 1):
            for i in (0, 5, W - 1):
                poses.append(((i + 0.5) * res, (j + 0.5) * res, 2 * math.pi * k / K))
                want.append(g[k, j, i])
    got = S.query(g, res, np.array(poses))
    assert np.max(np.abs(got[:, 0] - want)) < 1e-12


def test_query_exact_on_linear_fields():
    K, H, W, res = 5, 8, 10, 0.2
    k, j, i = np.meshgrid(np.arange(K), np.arange(H), np.arange(W), indexing="ij")
    g = 0.3 * i - 0.7 * j + 2.0                              # constant along yaw
    rng = np.random.default_rng(1)
    p = np.stack([rng.uniform(0.5 * res, (W - 0.5) * res, 50), rng.uniform(0.5 * res, (H - 0.5) * res, 50),
                  rng.uniform(-7, 7, 50)], 1)
    got = S.query(g, res, p)
    u, v = p[:, 0] / res - 0.5, p[:, 1] / res - 0.5
    assert np.max(np.abs(got[:, 0] - (0.3 * u - 0.7 * v + 2.0))) < 1e-12
    assert np.max(np.abs(got[:, 1] - 0.3 / res)) < 1e-12
    assert np.max(np.abs(got[:, 2] + 0.7 / res)) < 1e-12
    assert np.max(np.abs(got[:, 3])) < 1e-12


def test_query_yaw_wraps():
    g, res = grid_and_res()
    K = g.shape[0]
    base = np.array([[0.33, 0.41, 0.2], [0.5, 0.6, 2 * math.pi - 0.1], [0.7, 0.3, 2 * math.pi * (K - 0.5) / K]])
    a = S.query(g, res, base)
    b = S.query(g, res, base + np.array([0, 0, 2 * math.pi]))
    c = S.query(g, res, base - np.array([0, 0, 4 * math.pi]))
    assert np.max(np.abs(a - b)) < 1e-9 and np.max(np.abs(a - c)) < 1e-9
    # half way between the last bin and bin 0
    x, y = (3 + 0.5) * res, (2 + 0.5) * res
    v = S.query(g, res, np.array([[x, y, 2 * math.pi * (K - 0.5) / K]]))[0, 0]
    assert abs(v - 0.5 * (g[K - 1, 2, 3] + g[0, 2, 3])) < 1e-12


def test_query_gradients_match_finite_differences():
    g, res = grid_and_res()
    K, H, W = g.shape
    rng = np.random.default_rng(5)
    for _ in range(40):
        # interior points away from cell boundaries in every axis
        u = rng.integers(0, W - 1) + rng.uniform(0.2, 0.8)
        v = rng.integers(0, H - 1) + rng.uniform(0.2, 0.8)
        w = rng.integers(0, K) + rng.uniform(0.2, 0.8)
        p = np.array([(u + 0.5) * res, (v + 0.5) * res, w * 2 * math.pi / K])
        h = np.array([1e-5, 1e-5, 1e-5])
        got = S.query(g, res, p[None])[0]
        for a in range(3):
            e = np.zeros(3)
            e[a] = h[a]
            fd = (S.query(g, res, (p + e)[None])[0, 0] - S.query(g, res, (p - e)[None])[0, 0]) / (2 * h[a])
            assert abs(fd - got[1 + a]) < 1e-6 * max(1.0, abs(fd))


def test_query_clamps_outside_the_map():
    g, res = grid_and_res()
    K, H, W = g.shape
    inside = S.query(g, res, np.array([[0.5 * res, 3.2 * res, 0.4]]))[0]
    outside = S.query(g, res, np.array([[-2.0, 3.2 * res, 0.4]]))[0]
    assert abs(outside[0] - inside[0]) < 1e-12 and outside[1] == 0.0
    assert abs(outside[2] - inside[2]) < 1e-12 and abs(outside[3] - inside[3]) < 1e-12


def test_sampled_cells_match_whole_plane():
    rng = np.random.default_rng(9)
    obst = rng.random((37, 52)) < 0.07
    full = S.sdf_plane(obst, 0.1, 9)
    ys, xs = rng.integers(0, 37, 300), rng.integers(0, 52, 300)
    assert np.array_equal(S.sdf_cells(obst, 0.1, 9, ys, xs), full[ys, xs])
    none = np.zeros((5, 6), bool)
    assert np.all(S.sdf_cells(none, 0.1, 4, [0, 4], [0, 5]) == (4 - 0.5) * 0.1)
