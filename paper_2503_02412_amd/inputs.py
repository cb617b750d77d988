"""Seeded synthetic inputs shared by the oracle side and the GPU side.

This module holds workload definitions (map sizes, footprints, constants) and
terrain / trajectory generators.  It contains none of the assessment method's
arithmetic: no footprint tables, no fitting, no pose or risk maths.  Both the
CPU oracle (``oracle/``) and the HIP library (``paper_2503_02412_amd``) are fed
from here so that they see bit-identical inputs.

All draws come from ``numpy.random.Generator(PCG64(seed))`` in a fixed order.
The paper evaluates on an external procedural terrain generator and on real
terrain (Sec. VII-A); neither is available, so these generators stand in for
them, with the sizes and value ranges of the workloads listed below.

Map convention: ``H[iy, ix]`` row-major, float32, NaN = unknown; cell
``(ix, iy)`` has its centre at map-local metres ``((ix + 0.5) res, (iy + 0.5) res)``.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, asdict, replace

import numpy as np

# --------------------------------------------------------------------------
# Workload presets.  Constants follow the paper where it gives them
# (phi_x_max = phi_y_max = 0.52 rad, Sec. VII-B); the others (kappa_max,
# weights, r_max, min_valid) are not given by the paper and are parameters.
# --------------------------------------------------------------------------


@dataclass(frozen=True)
class Params:
    width: int
    height: int
    resolution: float
    n_yaw: int
    fp_length: float
    fp_width: float
    fp_nl: int
    fp_nw: int
    fp_shape: int = 0          # 0 = rectangle, 1 = inscribed ellipse mask
    kappa_max: float = 0.03
    phi_x_max: float = 0.52
    phi_y_max: float = 0.52
    w_kappa: float = 1.0 / 3.0
    w_phi_x: float = 1.0 / 3.0
    w_phi_y: float = 1.0 / 3.0
    risk_max: float = 0.5
    min_valid: int = 3
    precision: int = 0         # 0 = FP32, 1 = FP32 + FP64 for near-degenerate states
    fit: int = 0               # 0 = least-squares plane, 1 = principal-component plane

    def as_dict(self) -> dict:
        return asdict(self)

    def with_(self, **kw) -> "Params":
        return replace(self, **kw)

    @property
    def n_states(self) -> int:
        return self.width * self.height * self.n_yaw


# 64x64 @ 0.1 m, 16 yaw bins, 0.6 x 0.4 m footprint on a 6 x 4 sample grid.
CONFIG1 = Params(64, 64, 0.1, 16, 0.6, 0.4, 6, 4)
# 200x200 @ 0.1 m, 36 yaw bins, 1.0 x 0.6 m footprint on a 20 x 12 grid.
CONFIG2 = Params(200, 200, 0.1, 36, 1.0, 0.6, 20, 12)
# Rolling window: 400x400 @ 0.05 m, 72 yaw bins, 1.0 x 0.6 m on 20 x 12.
CONFIG3 = Params(400, 400, 0.05, 72, 1.0, 0.6, 20, 12)
# Large map: 800x800 @ 0.05 m, 72 yaw bins, 2.0 x 1.2 m on 40 x 24.
CONFIG5 = Params(800, 800, 0.05, 72, 2.0, 1.2, 40, 24)

PRESETS = {"config1": CONFIG1, "config2": CONFIG2, "config3": CONFIG3, "config5": CONFIG5}


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


# --------------------------------------------------------------------------
# G1: sum of 8 random-direction sinusoids plus Gaussian noise.
# --------------------------------------------------------------------------

def sinusoid_terrain(width: int, height: int, res: float, seed: int, *,
                     n_waves: int = 8, amp_max: float = 0.3,
                     wl_min: float = 1.0, wl_max: float = 6.0,
                     noise_sigma: float = 0.02) -> np.ndarray:
    rng = _rng(seed)
    alpha = rng.uniform(0.0, 2.0 * math.pi, n_waves)
    amp = rng.uniform(0.0, amp_max, n_waves)
    lam = rng.uniform(wl_min, wl_max, n_waves)
    psi = rng.uniform(0.0, 2.0 * math.pi, n_waves)
    noise = rng.normal(0.0, noise_sigma, (height, width))
    xs = (np.arange(width) + 0.5) * res
    ys = (np.arange(height) + 0.5) * res
    X, Y = np.meshgrid(xs, ys)
    h = np.zeros((height, width))
    for a, A, l, p in zip(alpha, amp, lam, psi):
        h += A * np.sin(2.0 * math.pi * (X * math.cos(a) + Y * math.sin(a)) / l + p)
    return (h + noise).astype(np.float32)


# --------------------------------------------------------------------------
# G2 / G3 / G5: fractal value noise + steps + NaN blobs.
# --------------------------------------------------------------------------

def _fade(t: np.ndarray) -> np.ndarray:
    return t * t * t * (t * (t * 6.0 - 15.0) + 10.0)


def value_noise(width: int, height: int, res: float, rng: np.random.Generator, *,
                octaves: int = 4, base: float = 3.2, lacunarity: float = 2.0,
                gain: float = 0.5) -> np.ndarray:
    xs = (np.arange(width) + 0.5) * res
    ys = (np.arange(height) + 0.5) * res
    out = np.zeros((height, width))
    spacing, amp = base, 1.0
    for _ in range(octaves):
        nxl = int(math.ceil(width * res / spacing)) + 2
        nyl = int(math.ceil(height * res / spacing)) + 2
        lat = rng.uniform(-1.0, 1.0, (nyl, nxl))
        gx = xs / spacing
        gy = ys / spacing
        ix = np.floor(gx).astype(np.int64)
        iy = np.floor(gy).astype(np.int64)
        tx = _fade(gx - ix)[None, :]
        ty = _fade(gy - iy)[:, None]
        v00 = lat[iy[:, None], ix[None, :]]
        v01 = lat[iy[:, None], ix[None, :] + 1]
        v10 = lat[iy[:, None] + 1, ix[None, :]]
        v11 = lat[iy[:, None] + 1, ix[None, :] + 1]
        top = v00 + (v01 - v00) * tx
        bot = v10 + (v11 - v10) * tx
        out += amp * (top + (bot - top) * ty)
        spacing /= lacunarity
        amp *= gain
    return out


def _max_slope(h: np.ndarray, res: float) -> float:
    gx = (h[1:-1, 2:] - h[1:-1, :-2]) / (2.0 * res)
    gy = (h[2:, 1:-1] - h[:-2, 1:-1]) / (2.0 * res)
    return float(np.sqrt(gx * gx + gy * gy).max())


def add_steps(h: np.ndarray, res: float, rng: np.random.Generator, n_steps: int = 4,
              lo: float = 0.1, hi: float = 0.3) -> np.ndarray:
    height, width = h.shape
    xs = (np.arange(width) + 0.5) * res
    ys = (np.arange(height) + 0.5) * res
    X, Y = np.meshgrid(xs, ys)
    for _ in range(n_steps):
        px = rng.uniform(0.0, width * res)
        py = rng.uniform(0.0, height * res)
        ang = rng.uniform(0.0, 2.0 * math.pi)
        dh = rng.uniform(lo, hi)
        side = (X - px) * math.cos(ang) + (Y - py) * math.sin(ang) > 0.0
        h = h + dh * side
    return h


def add_holes(h: np.ndarray, rng: np.random.Generator, frac: float, blob: int = 10) -> np.ndarray:
    """Punch NaN blobs of ``blob`` four-connected cells until >= frac is NaN."""
    height, width = h.shape
    mask = np.zeros((height, width), dtype=bool)
    target = int(math.ceil(frac * height * width))
    steps = ((1, 0), (-1, 0), (0, 1), (0, -1))
    count = 0
    while count < target:
        y0 = int(rng.integers(0, height))
        x0 = int(rng.integers(0, width))
        cells = [(y0, x0)]
        seen = {(y0, x0)}
        guard = 0
        while len(cells) < blob and guard < 1000:
            guard += 1
            cy, cx = cells[int(rng.integers(0, len(cells)))]
            dy, dx = steps[int(rng.integers(0, 4))]
            ny, nx = cy + dy, cx + dx
            if 0 <= ny < height and 0 <= nx < width and (ny, nx) not in seen:
                seen.add((ny, nx))
                cells.append((ny, nx))
        for cy, cx in cells:
            if not mask[cy, cx]:
                mask[cy, cx] = True
                count += 1
    out = h.copy()
    out[mask] = np.nan
    return out


def fractal_terrain(width: int, height: int, res: float, seed: int, *,
                    hole_frac: float = 0.05, max_slope_deg: float = 30.0,
                    n_steps: int = 4) -> np.ndarray:
    rng = _rng(seed)
    h = value_noise(width, height, res, rng)
    s = _max_slope(h, res)
    if s > 0:
        h = h * (math.tan(math.radians(max_slope_deg)) / s)
    h = add_steps(h, res, rng, n_steps=n_steps)
    if hole_frac > 0:
        h = add_holes(h, rng, hole_frac)
    return h.astype(np.float32)


# --------------------------------------------------------------------------
# Workload maps.
# --------------------------------------------------------------------------

def config1_map(seed: int = 1) -> np.ndarray:
    return sinusoid_terrain(64, 64, 0.1, seed)


def config2_map(seed: int = 2) -> np.ndarray:
    return fractal_terrain(200, 200, 0.1, seed, hole_frac=0.05)


def config5_map(seed: int = 5) -> np.ndarray:
    return fractal_terrain(800, 800, 0.05, seed, hole_frac=0.15)


def trajectory(seed: int = 3, n_steps: int = 100, step_m: float = 0.5) -> np.ndarray:
    """Robot (x, y) positions in metres: start at 0, then n_steps moves of
    step_m in a uniformly random heading.  Returns (n_steps + 1, 2) float64."""
    rng = _rng(seed)
    heading = rng.uniform(0.0, 2.0 * math.pi, n_steps)
    pos = np.zeros((n_steps + 1, 2))
    pos[1:, 0] = np.cumsum(step_m * np.cos(heading))
    pos[1:, 1] = np.cumsum(step_m * np.sin(heading))
    return pos


@dataclass
class World:
    """A large world height grid in which a rolling window moves.

    World cell (gx, gy) has its centre at ((gx + 0.5) res, (gy + 0.5) res)
    metres, and is stored at ``heights[gy - gy0, gx - gx0]``."""
    heights: np.ndarray
    gx0: int
    gy0: int
    res: float

    def window(self, ox: int, oy: int, w: int, h: int) -> np.ndarray:
        """Heights of world cells [ox, ox+w) x [oy, oy+h); NaN outside the grid."""
        out = np.full((h, w), np.nan, dtype=np.float32)
        ys0, xs0 = oy - self.gy0, ox - self.gx0
        H, W = self.heights.shape
        y_lo, y_hi = max(0, ys0), min(H, ys0 + h)
        x_lo, x_hi = max(0, xs0), min(W, xs0 + w)
        if y_lo < y_hi and x_lo < x_hi:
            out[y_lo - ys0:y_hi - ys0, x_lo - xs0:x_hi - xs0] = self.heights[y_lo:y_hi, x_lo:x_hi]
        return out


def rolling_world(params: Params = CONFIG3, seed: int = 3, n_steps: int = 100,
                  hole_frac: float = 0.05) -> tuple[World, np.ndarray]:
    """World grid covering the whole seeded trajectory plus one window of margin
    on every side, built with the fractal generator at the window's resolution."""
    traj = trajectory(seed, n_steps)
    res = params.resolution
    margin = max(params.width, params.height)
    gx_lo = int(math.floor(traj[:, 0].min() / res)) - margin
    gx_hi = int(math.floor(traj[:, 0].max() / res)) + margin
    gy_lo = int(math.floor(traj[:, 1].min() / res)) - margin
    gy_hi = int(math.floor(traj[:, 1].max() / res)) + margin
    w, h = gx_hi - gx_lo + 1, gy_hi - gy_lo + 1
    heights = fractal_terrain(w, h, res, seed + 1000, hole_frac=hole_frac,
                              n_steps=4 * max(1, (w * h) // (400 * 400)))
    return World(heights, gx_lo, gy_lo, res), traj


# --------------------------------------------------------------------------
# Learned-surrogate data: config-1-style sinusoid terrains (64 x 64 @ 0.1 m)
# with two step lines and 5% unknown blobs, labelled by the plain method with
# the 200 x 200 workload's footprint (1.0 x 0.6 m on 20 x 12) and 36 yaw bins.
# --------------------------------------------------------------------------

SURROGATE_LABEL_PARAMS = CONFIG2.with_(width=64, height=64)
# The same map with a 2.0 x 1.2 m footprint on 40 x 24 samples: four times the
# plain method's work per state, still inside the network's 24 x 24 window.
CONFIG2_LARGE_FOOTPRINT = CONFIG2.with_(fp_length=2.0, fp_width=1.2, fp_nl=40, fp_nw=24)
SURROGATE_TRAIN_SEEDS = tuple(range(1000, 1070))
SURROGATE_VAL_SEEDS = (1070, 1071)
SURROGATE_EVAL_SEEDS = (2000, 2001, 2002, 2003)


def surrogate_training_map(seed: int, size: int = 64, res: float = 0.1) -> np.ndarray:
    rng = _rng(seed)
    h = sinusoid_terrain(size, size, res, seed + 50000).astype(np.float64)
    h = add_steps(h, res, rng, n_steps=2)
    h = add_holes(h, rng, 0.05)
    return h.astype(np.float32)


def surrogate_samples(n_maps: int, size: int, n_yaw: int, seed: int, count: int | None = None,
                      margin: int = 0) -> np.ndarray:
    """All (map, cy, cx, k) with the cell at least `margin` cells inside the map
    (windows may extend past the edge), in a seeded random order (first
    `count` kept); int32 [count, 4]."""
    c = np.arange(margin, size - margin)
    m, y, x, k = np.meshgrid(np.arange(n_maps), c, c, np.arange(n_yaw), indexing="ij")
    s = np.stack([m.ravel(), y.ravel(), x.ravel(), k.ravel()], 1).astype(np.int32)
    perm = _rng(seed).permutation(len(s))
    s = s[perm]
    return s if count is None else s[:count]


# --------------------------------------------------------------------------
# Planner-side fields: status bytes and query poses.  The status bits are those
# of the library's output (1 valid, 2 curvature obstacle, 4 tilt obstacle,
# 8 near-degenerate, 16 traversable, 32 surrogate); here they are drawn as
# shapes, not computed from terrain.
# --------------------------------------------------------------------------


def synthetic_status(width: int, height: int, n_yaw: int, seed: int, *,
                     n_obstacles: int | None = None, n_unknown: int | None = None,
                     max_radius: int = 9) -> np.ndarray:
    """uint8 [K][H][W] status planes: elliptical obstacle blobs whose extent
    changes with the yaw bin (obstacles of a yawed footprint grow along the
    body's long axis), tagged curvature, tilt, both, or surrogate-answered
    and not traversable; elliptical unknown patches shared by every yaw bin;
    and random near-degenerate / traversable bits elsewhere, with the
    surrogate bit only on traversable states there."""
    rng = _rng(seed)
    area = width * height
    n_obstacles = max(1, area // 700) if n_obstacles is None else n_obstacles
    n_unknown = max(1, area // 2500) if n_unknown is None else n_unknown

    def blobs(n):
        return (rng.uniform(0, width, n), rng.uniform(0, height, n),
                rng.uniform(0.5, max_radius, n), rng.uniform(0.5, max_radius, n),
                rng.uniform(0, math.pi, n))

    unknown = np.zeros((height, width), dtype=bool)
    for cx, cy, ra, rb, ang in zip(*blobs(n_unknown)):
        e = _ellipse(unknown.shape, cx, cy, ra, rb, ang)
        if e is not None:
            unknown[e[0]] |= e[1]
    ox, oy, oa, ob, oang = blobs(n_obstacles)
    kind = rng.integers(0, 4, n_obstacles)      # curvature, tilt, both, surrogate
    extra = rng.integers(0, 64, (n_yaw, height, width)).astype(np.uint8) & (8 | 16 | 32)
    extra |= (extra & 32) >> 1                  # a free surrogate answer is traversable
    out = np.empty((n_yaw, height, width), dtype=np.uint8)
    for k in range(n_yaw):
        th = 2.0 * math.pi * k / n_yaw
        bits = np.zeros((height, width), dtype=np.uint8)
        for i in range(n_obstacles):
            grow = 1.0 + 0.5 * abs(math.cos(th - oang[i]))
            e = _ellipse(bits.shape, ox[i], oy[i], oa[i] * grow, ob[i], th)
            if e is not None:
                bits[e[0]] |= np.where(e[1], (2, 4, 6, 32)[kind[i]], 0).astype(np.uint8)
        plane = np.where(bits != 0, 1 | bits, 1 | extra[k]).astype(np.uint8)
        plane[bits != 0] |= extra[k][bits != 0] & 8
        plane[unknown] = extra[k][unknown] & 8
        out[k] = plane
    return out


def _ellipse(shape, cx: float, cy: float, ra: float, rb: float, ang: float):
    """(window slices, boolean mask over the window) of the cells whose centres
    lie in the rotated ellipse, or None if the window is empty."""
    height, width = shape
    r = int(math.ceil(max(ra, rb))) + 1
    x0, x1 = max(0, int(cx) - r), min(width, int(cx) + r + 1)
    y0, y1 = max(0, int(cy) - r), min(height, int(cy) + r + 1)
    if x0 >= x1 or y0 >= y1:
        return None
    ys, xs = np.mgrid[y0:y1, x0:x1]
    dx, dy = xs + 0.5 - cx, ys + 0.5 - cy
    c, s = math.cos(ang), math.sin(ang)
    u, v = dx * c + dy * s, -dx * s + dy * c
    return (slice(y0, y1), slice(x0, x1)), (u / ra) ** 2 + (v / rb) ** 2 <= 1.0


def query_poses(n: int, width: int, height: int, res: float, seed: int,
                margin_cells: float = 3.0) -> np.ndarray:
    """float32 [n][3] poses (x, y, theta): positions uniform over the map plus a
    margin on every side (so some fall outside and are clamped), yaw uniform
    over several turns either way."""
    rng = _rng(seed)
    x = rng.uniform(-margin_cells * res, (width + margin_cells) * res, n)
    y = rng.uniform(-margin_cells * res, (height + margin_cells) * res, n)
    th = rng.uniform(-6.0 * math.pi, 6.0 * math.pi, n)
    return np.stack([x, y, th], 1).astype(np.float32)


def trajectory_query_poses(n_traj: int, n_per: int, width: int, height: int, res: float,
                           seed: int) -> np.ndarray:
    """float32 [n_traj * n_per][3] poses sampled along smooth paths, the way a
    trajectory optimiser reads the fields: each path starts at a uniform
    position with a uniform heading, turns at a constant curvature drawn from
    [-1, 1] 1/m and advances half a cell per sample; theta is the heading."""
    rng = _rng(seed)
    x0 = rng.uniform(0.0, width * res, n_traj)[:, None]
    y0 = rng.uniform(0.0, height * res, n_traj)[:, None]
    h0 = rng.uniform(-math.pi, math.pi, n_traj)[:, None]
    kap = rng.uniform(-1.0, 1.0, n_traj)[:, None]
    s = (np.arange(n_per) * 0.5 * res)[None, :]
    th = h0 + kap * s
    # closed form of the arc (straight-line limit for tiny curvature)
    small_k = np.abs(kap) < 1e-9
    safe_k = np.where(small_k, 1.0, kap)
    x = np.where(small_k, x0 + s * np.cos(h0), x0 + (np.sin(th) - np.sin(h0)) / safe_k)
    y = np.where(small_k, y0 + s * np.sin(h0), y0 - (np.cos(th) - np.cos(h0)) / safe_k)
    return np.stack([x.ravel(), y.ravel(), th.ravel()], 1).astype(np.float32)


# --------------------------------------------------------------------------
# Elevation-map update: synthetic LiDAR scans.  Points are drawn on a terrain
# around the robot and expressed in the sensor frame; no occlusion is modelled.
# --------------------------------------------------------------------------


def rotation_zyx(yaw: float, pitch: float, roll: float) -> np.ndarray:
    """Rz(yaw) Ry(pitch) Rx(roll), float64 [3][3]."""
    cy, sy = math.cos(yaw), math.sin(yaw)
    cp, sp = math.cos(pitch), math.sin(pitch)
    cr, sr = math.cos(roll), math.sin(roll)
    Rz = np.array([[cy, -sy, 0.0], [sy, cy, 0.0], [0.0, 0.0, 1.0]])
    Ry = np.array([[cp, 0.0, sp], [0.0, 1.0, 0.0], [-sp, 0.0, cp]])
    Rx = np.array([[1.0, 0.0, 0.0], [0.0, cr, -sr], [0.0, sr, cr]])
    return Rz @ Ry @ Rx


def synthetic_scan(terrain: np.ndarray, res: float, n_points: int, seed: int, *,
                   robot_xy=None, max_range: float = 8.0, canopy_frac: float = 0.03,
                   stray_frac: float = 0.02, origin=(0, 0)) -> dict:
    """A scan of `terrain` (float32 [H][W], NaN = no return; cell (i, j) of the
    array is world cell (origin_x + i, origin_y + j)) seen from a robot at
    robot_xy (world metres; default: the terrain's centre).  Ranges
    0.3 + (max_range - 0.3) u^2 (denser near the sensor), azimuth uniform,
    height = the terrain cell's height + N(0, 0.01^2); a fraction of points
    lies 1-2.5 m above the ground (overhangs), another 4-10 m above (outside
    any height band).  Returns the points (float32 [n][3], sensor frame; rays
    onto unknown cells or off the terrain give no point) and the frames and
    noise model of the scan."""
    rng = _rng(seed)
    Ht, Wt = terrain.shape
    ox, oy = origin
    if robot_xy is None:
        robot_xy = ((ox + Wt / 2.0) * res, (oy + Ht / 2.0) * res)
    rx, ry = robot_xy
    yaw = rng.uniform(-math.pi, math.pi)
    pitch, roll = rng.normal(0.0, 0.05, 2)
    R_B = rotation_zyx(yaw, pitch, roll)
    ci = min(max(int(math.floor(rx / res)) - ox, 0), Wt - 1)
    cj = min(max(int(math.floor(ry / res)) - oy, 0), Ht - 1)
    ground = float(terrain[cj, ci]) if np.isfinite(terrain[cj, ci]) else 0.0
    p_B = np.array([rx, ry, ground + 0.4])
    R_BS = rotation_zyx(0.02, -0.03, 0.01)
    p_BS = np.array([0.15, 0.0, 0.35])
    r = 0.3 + (max_range - 0.3) * rng.random(n_points) ** 2
    a = rng.uniform(0.0, 2.0 * math.pi, n_points)
    wx = rx + r * np.cos(a)
    wy = ry + r * np.sin(a)
    i = np.floor(wx / res).astype(np.int64) - ox
    j = np.floor(wy / res).astype(np.int64) - oy
    inside = (i >= 0) & (i < Wt) & (j >= 0) & (j < Ht)
    z = np.full(n_points, np.nan)
    z[inside] = terrain[j[inside], i[inside]]
    z = z + rng.normal(0.0, 0.01, n_points)
    u = rng.random(n_points)
    z = np.where(u < canopy_frac, z + rng.uniform(1.0, 2.5, n_points), z)
    z = np.where((u >= canopy_frac) & (u < canopy_frac + stray_frac),
                 z + rng.uniform(4.0, 10.0, n_points), z)
    ok = np.isfinite(z)
    P = np.stack([wx[ok], wy[ok], z[ok]], 1)
    # sensor frame: R_BS^T (R_B^T (P - p_B) - p_BS)
    body = (P - p_B) @ R_B
    sensor = (body - p_BS) @ R_BS
    return {
        "points": sensor.astype(np.float32),
        "R_B": R_B, "p_B": p_B, "R_BS": R_BS, "p_BS": p_BS,
        "Sigma_R": np.diag([0.002 ** 2, 0.002 ** 2, 0.004 ** 2]),
        "Sigma_B": np.diag([0.01 ** 2, 0.01 ** 2, 0.02 ** 2]),
        "sigma_range": 0.02, "sigma_angle": 0.002,
        "z_min": -3.0, "z_max": 2.0, "mahalanobis": 3.0,
    }
