"""Pins of the FP64 elevation-update reference (oracle/elevation.py): closed
forms of the point variance, a Monte-Carlo check of Eq. 5-9 under the stated
perturbation model, the Kalman and Mahalanobis rules, and nearest-neighbour
inpainting against scipy's exact distance transform."""
import math

import numpy as np
import pytest
from scipy import ndimage
from scipy.spatial.transform import Rotation

from oracle import elevation as E

I3 = np.eye(3)
Z3 = np.zeros((3, 3))


def run(points, R_B=I3, p_B=(0, 0, 0), R_BS=I3, p_BS=(0, 0, 0), Sigma_R=Z3, Sigma_B=Z3,
        s_r=0.02, s_a=0.001, z_min=-10.0, z_max=10.0, res=0.1, W=100, H=100, ox=-50, oy=-50):
    return E.process_points(points, R_B, p_B, R_BS, p_BS, Sigma_R, Sigma_B, s_r, s_a, z_min, z_max,
                            res, W, H, ox, oy)


def test_variance_closed_forms():
    pts = np.array([[0.0, 0.0, -2.0], [3.0, 0.0, 0.0], [0.0, 4.0, 0.0]])
    SB = np.diag([1e-4, 2e-4, 3e-4])
    cell, z, var = run(pts, p_BS=(0, 0, 1.0), Sigma_B=SB)
    # straight down: range noise only; horizontal: angular noise times range
    np.testing.assert_allclose(var, [0.02 ** 2 + 3e-4, (0.001 * 3) ** 2 + 3e-4,
                                     (0.001 * 4) ** 2 + 3e-4], rtol=1e-12)
    np.testing.assert_allclose(z, [-1.0, 1.0, 1.0], atol=1e-15)
    # a small rotation about body y moves the point at x = 3 (z = 1) by -3 d in height
    SR = np.diag([1e-4, 4e-4, 9e-4])
    _, _, var2 = run(pts[1:2], p_BS=(0, 0, 1.0), Sigma_R=SR, s_r=0.0, s_a=0.0)
    np.testing.assert_allclose(var2, [9 * 4e-4], rtol=1e-12)


def test_variance_matches_monte_carlo():
    """Sample the sensor noise, a body-frame rotation perturbation R_B Exp(d)
    and a position perturbation, push the point through exactly, and compare
    the sample variance of its height with Eq. 5-9."""
    rng = np.random.default_rng(7)
    R_B = Rotation.from_rotvec([0.2, -0.35, 1.1]).as_matrix()
    R_BS = Rotation.from_rotvec([-0.1, 0.25, 0.4]).as_matrix()
    p_B, p_BS = np.array([1.0, -2.0, 0.5]), np.array([0.2, 0.1, 0.6])
    A = rng.normal(size=(3, 3)) * 0.01
    SR = A @ A.T + np.diag([1e-5, 2e-5, 3e-5])
    B = rng.normal(size=(3, 3)) * 0.02
    SB = B @ B.T
    s_r, s_a = 0.03, 0.004
    pts = np.array([[4.0, 1.0, -1.5], [-2.0, 6.0, 0.5], [0.5, -0.3, -3.0]])
    _, z0, var = run(pts, R_B, p_B, R_BS, p_BS, SR, SB, s_r, s_a)
    n = 400_000
    for i, p in enumerate(pts):
        r = np.linalg.norm(p)
        u = p / r
        SS = s_r ** 2 * np.outer(u, u) + (s_a * r) ** 2 * (I3 - np.outer(u, u))
        eps_s = rng.multivariate_normal(np.zeros(3), SS, n)
        d = rng.multivariate_normal(np.zeros(3), SR, n)
        eps_b = rng.multivariate_normal(np.zeros(3), SB, n)
        Rp = R_B @ Rotation.from_rotvec(d).as_matrix()              # [n, 3, 3]
        q = (R_BS @ (p + eps_s).T).T + p_BS
        z = np.einsum("j,njk,nk->n", np.array([0.0, 0.0, 1.0]), Rp, q) + p_B[2] + eps_b[:, 2]
        assert abs(z.mean() - z0[i]) < 5 * math.sqrt(var[i] / n) + 1e-6
        assert abs(z.var() / var[i] - 1.0) < 0.015, (i, z.var(), var[i])


def test_cells_frames_and_filters():
    R_B = Rotation.from_euler("z", 90, degrees=True).as_matrix()
    # sensor point (1, 0, 0) -> body (1, 0, 0) -> map (0, 1, 0) + p_B
    p_B = (2.07, 3.03, 0.0)
    pts = np.array([[1.0, 0.0, 0.0],       # -> (2.07, 4.03): world cell (20, 40)
                    [1.0, 0.0, 5.0],       # body z 5 > z_max: dropped
                    [-30.0, 0.0, 0.0],     # far outside the window: dropped
                    [np.nan, 0.0, 0.0]])   # not a point: dropped
    cell, z, _ = run(pts, R_B=R_B, p_B=p_B, z_max=2.0, W=30, H=20, ox=10, oy=30)
    assert cell[0] == (40 - 30) * 30 + (20 - 10)
    assert list(cell[1:]) == [-1, -1, -1]
    assert abs(z[0] - 0.0) < 1e-15
    # the band is in the body frame: a robot 3 m up keeps its own ground points
    # (map height 3 > z_max) and drops a point 3 m below it (map height 0)
    cell, z, _ = run(pts[:1].repeat(2, 0) + [[0, 0, 0], [0, 0, -3.0]], R_B=R_B,
                     p_B=(2.07, 3.03, 3.0), z_min=-2.0, z_max=2.0, W=30, H=20, ox=10, oy=30)
    assert cell[0] >= 0 and cell[1] == -1 and abs(z[0] - 3.0) < 1e-15


def fuse_one(h0, v0, zs, ss, tau=3.0):
    Hm = np.array([[h0]], np.float32)
    Vm = np.array([[v0]], np.float32)
    return E.fuse(Hm, Vm, np.zeros(len(zs), np.int64), np.array(zs, float), np.array(ss, float), tau)


def test_fusion_rules():
    h, v, used = fuse_one(np.nan, 0.0, [1.5], [0.01])
    assert (h[0, 0], v[0, 0], used) == (np.float32(1.5), np.float32(0.01), 1)
    # two consistent points: information-weighted mean
    h, v, _ = fuse_one(np.nan, 0.0, [1.0, 1.02], [0.01, 0.03])
    want_v = 1.0 / (1 / 0.01 + 1 / 0.03)
    want_h = want_v * (1.0 / 0.01 + 1.02 / 0.03)
    assert h[0, 0] == np.float32(want_h) and v[0, 0] == np.float32(want_v)
    # a prior estimate and a consistent point
    h, v, _ = fuse_one(2.0, 0.04, [2.1], [0.01])
    assert h[0, 0] == np.float32((0.04 * 2.1 + 0.01 * 2.0) / 0.05)
    assert v[0, 0] == np.float32(0.04 * 0.01 / 0.05)
    # a higher outlier replaces the cell, a lower one is dropped
    h, v, used = fuse_one(1.0, 0.0001, [1.5], [0.02])
    assert (h[0, 0], v[0, 0], used) == (np.float32(1.5), np.float32(0.02), 1)
    h, v, used = fuse_one(1.0, 0.0001, [0.5], [0.02])
    assert (h[0, 0], v[0, 0], used) == (np.float32(1.0), np.float32(0.0001), 0)
    # exactly at the gate: fused, not an outlier
    h, v, used = fuse_one(0.0, 1.0, [3.0], [1.0])
    assert used == 1 and h[0, 0] == np.float32(1.5)


def test_fusion_of_consistent_points_is_batch_estimate():
    rng = np.random.default_rng(3)
    zs = 0.7 + rng.normal(0, 0.01, 50)
    ss = rng.uniform(0.5e-4, 2e-4, 50)
    h, v, used = fuse_one(np.nan, 0.0, zs, ss, tau=1e6)
    w = 1.0 / ss
    assert used == 50
    assert abs(h[0, 0] - np.sum(w * zs) / np.sum(w)) < 1e-6
    assert abs(v[0, 0] / (1.0 / np.sum(w)) - 1) < 1e-6


def test_fusion_order_and_cells():
    Hm = np.full((2, 3), np.nan, np.float32)
    Vm = np.zeros((2, 3), np.float32)
    cell = np.array([4, 1, 4, -1, 4])
    z = np.array([1.0, 2.0, 3.0, 9.0, 1.1])
    s = np.array([0.01, 0.01, 0.01, 0.01, 0.01])
    h, v, used = E.fuse(Hm, Vm, cell, z, s, 3.0)
    # cell 4 sees 1.0, then 3.0 (a higher outlier: replaces), then 1.1 (a lower outlier: dropped)
    assert h.flat[4] == np.float32(3.0) and h.flat[1] == np.float32(2.0)
    assert np.isnan(h.flat[0]) and used == 3


def test_inpaint_matches_exact_distance_transform():
    rng = np.random.default_rng(11)
    h = rng.normal(size=(37, 53)).astype(np.float32)
    hole = rng.random(h.shape) < 0.35
    hole[10:25, 20:40] = True
    h[hole] = np.nan
    h[0, 0] = np.inf
    radius = 6
    out = E.inpaint_nearest(h, radius)
    known = np.isfinite(h)
    assert np.array_equal(out[known], h[known])
    dist = ndimage.distance_transform_edt(~known)
    filled = ~known & (dist <= radius)
    assert np.all(np.isfinite(out[filled])) and np.all(np.isnan(out[~known & ~filled]))
    # the value comes from a known cell at exactly the nearest distance
    ky, kx = np.nonzero(known)
    for y, x in zip(*np.nonzero(filled)):
        d2 = (ky - y) ** 2 + (kx - x) ** 2
        at = d2 == round(dist[y, x] ** 2)
        assert out[y, x] in set(h[ky[at], kx[at]].tolist())


def test_inpaint_tie_break():
    h = np.full((5, 5), np.nan, np.float32)
    h[1, 2], h[3, 2] = 1.0, 2.0          # dy = -1 and +1: the smaller dy wins
    h[2, 1], h[2, 3] = 3.0, 4.0          # also at distance 1, dy = 0: beats dy = +1 only
    out = E.inpaint_nearest(h, 2)
    assert out[2, 2] == np.float32(1.0)
    h[1, 2] = np.nan
    out = E.inpaint_nearest(h, 2)
    assert out[2, 2] == np.float32(3.0)  # dy = 0, dx = -1 before dx = +1 and dy = +1


def ray(H, sensor, pts_map, margin=0.0, res=0.1, ox=0, oy=0):
    """Identity frames: the robot (and sensor) at `sensor`, points given in
    map coordinates."""
    pts = np.asarray(pts_map, dtype=np.float64) - np.asarray(sensor)
    return E.raycast_reset(H, pts, I3, sensor, I3, (0, 0, 0), res, ox, oy, margin)


def test_raycast_level_ray():
    H = np.full((3, 12), 0.5, np.float32)
    H[0, 3] = H[0, 7] = H[0, 10] = 2.0
    out, n = ray(H, (0.05, 0.05, 1.0), [[1.05, 0.05, 1.0]])
    assert n == 2 and np.isnan(out[0, 3]) and np.isnan(out[0, 7])
    assert out[0, 10] == 2.0                           # the point's own cell is kept
    assert np.array_equal(out[1:], H[1:])


def test_raycast_sloped_ray_threshold_and_margin():
    # from z = 2 at x = 0.05 down to z = 0 at x = 1.05: the ray is highest where
    # it enters cell i, at 2.1 - 0.2 i (cell 0: 2.0, where it starts)
    H = np.full((1, 12), -5.0, np.float32)
    top = [2.0] + [2.1 - 0.2 * i for i in range(1, 10)]
    for i in range(10):
        H[0, i] = top[i] + (0.01 if i % 2 else -0.01)
    out, n = ray(H, (0.05, 0.05, 2.0), [[1.05, 0.05, 0.0]])
    assert n == 5 and all(np.isnan(out[0, i]) == bool(i % 2) for i in range(10))
    out, n = ray(H, (0.05, 0.05, 2.0), [[1.05, 0.05, 0.0]], margin=0.02)
    assert n == 0


def test_raycast_corner_touch_and_vertical_ray():
    H = np.full((6, 6), 5.0, np.float32)
    out, n = ray(H, (0.05, 0.05, 1.0), [[0.35, 0.35, 1.0]])
    # the diagonal passes the corners exactly: only (0,0), (1,1), (2,2) are crossed;
    # (3,3) is the point's own cell
    reset = np.isnan(out)
    assert n == 3 and reset[0, 0] and reset[1, 1] and reset[2, 2] and reset.sum() == 3
    out, n = ray(H, (0.05, 0.05, 1.0), [[0.05, 0.55, 1.0]])
    assert n == 5 and np.isnan(out[:5, 0]).all() and out[5, 0] == 5.0


def test_raycast_matches_dense_sampling():
    """One random ray at a time against the segment sampled densely: a crossed
    cell standing clearly above the sampled ray is reset, one below is not."""
    rng = np.random.default_rng(21)
    res, Hn, Wn = 0.1, 30, 40
    for _ in range(60):
        H = rng.uniform(-1.0, 1.0, (Hn, Wn)).astype(np.float32)
        s = (rng.uniform(0.5, 3.5), rng.uniform(0.5, 2.5), rng.uniform(-0.5, 1.0))
        e = (rng.uniform(0.0, 4.0), rng.uniform(0.0, 3.0), rng.uniform(-1.0, 0.5))
        out, _ = ray(H, s, [e])
        t = np.linspace(0.0, 1.0, 40001)
        x = s[0] + t * (e[0] - s[0])
        y = s[1] + t * (e[1] - s[1])
        z = s[2] + t * (e[2] - s[2])
        ci, cj = np.floor(x / res).astype(int), np.floor(y / res).astype(int)
        own = (math.floor(e[0] / res), math.floor(e[1] / res))
        zs = {}
        for i, j, zz in zip(ci, cj, z):
            if (i, j) != own and 0 <= i < Wn and 0 <= j < Hn:
                zs[(i, j)] = max(zs.get((i, j), -np.inf), zz)
        slack = abs(e[2] - s[2]) / 40000 + 1e-9
        for (i, j), zz in zs.items():
            if H[j, i] > zz + slack:
                assert np.isnan(out[j, i])
            elif H[j, i] < zz:
                assert out[j, i] == H[j, i]
        untouched = np.ones((Hn, Wn), bool)
        for (i, j) in zs:
            untouched[j, i] = False
        # a cell the samples never entered is crossed for less than 1/40000 of the ray
        assert np.isnan(out[untouched]).sum() <= 2


def test_raycast_sensor_cell_and_mounting():
    # the ray starts at the sensor: in the sensor's own cell it is highest at t = 0
    H = np.full((1, 12), -5.0, np.float32)
    H[0, 0] = 2.05
    out, n = ray(H, (0.05, 0.05, 2.0), [[1.05, 0.05, 0.0]])
    assert n == 1 and np.isnan(out[0, 0])
    # the sensor sits at R_B p_BS + p_B: a robot turned by 90 degrees with the
    # sensor mounted 0.5 m to its left puts it at (0.05, 0.05, 1.0)
    R_B = Rotation.from_euler("z", 90, degrees=True).as_matrix()
    p_B, p_BS = np.array([0.55, 0.05, 0.0]), np.array([0.0, 0.5, 1.0])
    P = np.array([[1.05, 0.05, 1.0]])
    pts = (P - p_B) @ R_B - p_BS                      # sensor frame, with R_BS = I
    H = np.full((3, 12), 0.5, np.float32)
    H[0, 3] = H[0, 7] = H[0, 10] = 2.0
    out, n = E.raycast_reset(H, pts, R_B, p_B, I3, p_BS, 0.1, 0, 0, 0.0)
    assert n == 2 and np.isnan(out[0, 3]) and np.isnan(out[0, 7]) and out[0, 10] == 2.0
