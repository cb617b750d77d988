"""FP64 reference of the SE(2) signed distance field and the trilinear
Risk / SDF query -- TEST INFRASTRUCTURE.

Only the test-suite, the smoke check and the CPU-baseline leg of the benchmark
may import this module.  It shares no code with the library.

What it computes (the paper's planner-side use of the risk map, Sec. V and
Sec. VI-B/VI-C): the SDF G_c over SE(2) states is, at each state, the distance
to the edge of the nearest obstacle region, negative inside obstacles; the
planner reads G_c and Risk at arbitrary poses by trilinear interpolation, with
the yaw axis handled on SO(2).

Readings (the paper leaves these open; the same readings are used by the
library):
  - obstacle states: the explicit obstacles of Algorithm 1 (curvature or tilt
    early-out, status bits 2 and 4), states answered by the learned surrogate
    (bit 32) without the traversable bit (16) -- the network does not say
    which early-out applies, so its non-traversable answers all count, the
    safe side -- and, when `unknown_is_obstacle`, the UNKNOWN states (status
    bit 1 clear);
  - distance: Euclidean, within each yaw bin's (x, y) plane, between cell
    centres, in metres; for a free state the distance to the nearest obstacle
    state, for an obstacle state the distance to the nearest free state; the
    edge between two cells lies half a cell from each centre, so
        G = +(d_obstacle - res / 2)  for free states,
        G = -(d_free     - res / 2)  for obstacle states;
  - distances are capped: d is replaced by min(d, cap * res) with cap an
    integer number of cells (no obstacle / no free state in the plane gives
    the capped value too);
  - query frame: logical map coordinates in metres with the corner of cell
    (0, 0) at the origin, so cell (i, j)'s centre is ((i + 0.5) res,
    (j + 0.5) res); yaw bin k sits at 2 pi k / K.  A pose outside the cell
    centres' range is clamped onto it (the value of the clamped point, and a
    zero derivative along the clamped axis); the yaw wraps.  Derivatives are
    those of the interpolant inside the cell [floor, floor + 1] of each axis.
"""
from __future__ import annotations

import math

import numpy as np

VALID, CURV, TILT, TRAV, SURROGATE = 1, 2, 4, 16, 32


def obstacle_mask(status: np.ndarray, unknown_is_obstacle: bool = True) -> np.ndarray:
    st = np.asarray(status).astype(np.int64)
    m = (st & (CURV | TILT)) != 0
    m |= ((st & SURROGATE) != 0) & ((st & TRAV) == 0)
    if unknown_is_obstacle:
        m |= (st & VALID) == 0
    return m


def sdf_plane(obst: np.ndarray, res: float, cap: int) -> np.ndarray:
    """Signed distance of one [H][W] plane by brute force over all cell pairs."""
    H, W = obst.shape
    ys, xs = np.mgrid[0:H, 0:W]
    pts = np.stack([xs.ravel(), ys.ravel()], 1).astype(np.float64)
    o = obst.ravel()
    out = np.empty(H * W)
    for target, sign, sel in ((o, 1.0, ~o), (~o, -1.0, o)):
        tgt = pts[target]
        idx = np.nonzero(sel)[0]
        if idx.size == 0:
            continue
        if tgt.shape[0] == 0:
            d = np.full(idx.size, float(cap))
        else:
            d = np.empty(idx.size)
            for a in range(0, idx.size, 2048):
                q = pts[idx[a:a + 2048]]
                diff = q[:, None, :] - tgt[None, :, :]
                d[a:a + 2048] = np.sqrt(np.min(np.sum(diff * diff, axis=2), axis=1))
            d = np.minimum(d, float(cap))
        out[idx] = sign * (d - 0.5) * res
    return out.reshape(H, W)


def sdf_cells(obst: np.ndarray, res: float, cap: int, ys, xs) -> np.ndarray:
    """Signed distance of the listed cells (ys[i], xs[i]) of one [H][W] plane,
    each by brute force over every cell of the plane (for sampled checks of
    large maps)."""
    H, W = obst.shape
    gy, gx = np.mgrid[0:H, 0:W]
    out = np.empty(len(ys))
    for n, (y, x) in enumerate(zip(ys, xs)):
        inside = bool(obst[y, x])
        tgt = ~obst if inside else obst
        if not tgt.any():
            d = float(cap)
        else:
            d = min(math.sqrt(float(np.min((gx[tgt] - x) ** 2 + (gy[tgt] - y) ** 2))), float(cap))
        out[n] = (-1.0 if inside else 1.0) * (d - 0.5) * res
    return out


def sdf_planes(status: np.ndarray, res: float, cap: int, unknown_is_obstacle: bool = True):
    """SDF of every yaw plane of status [K][H][W] (logical layout)."""
    obst = obstacle_mask(status, unknown_is_obstacle)
    return np.stack([sdf_plane(obst[k], res, cap) for k in range(obst.shape[0])])


def query(grid: np.ndarray, res: float, poses: np.ndarray):
    """Trilinear interpolation of grid [K][H][W] at poses [n][3] = (x, y,
    theta); returns value, d/dx, d/dy, d/dtheta per pose ([n][4])."""
    K, H, W = grid.shape
    out = np.zeros((len(poses), 4))
    dth = 2.0 * math.pi / K
    for n, (x, y, th) in enumerate(np.asarray(poses, dtype=np.float64)):
        u = min(max(x / res - 0.5, 0.0), W - 1.0)
        v = min(max(y / res - 0.5, 0.0), H - 1.0)
        inside_u = 0.0 <= x / res - 0.5 <= W - 1.0
        inside_v = 0.0 <= y / res - 0.5 <= H - 1.0
        w = (th / dth) % K
        i0 = min(int(math.floor(u)), W - 2) if W > 1 else 0
        j0 = min(int(math.floor(v)), H - 2) if H > 1 else 0
        k0 = int(math.floor(w)) % K
        fu, fv, fw = u - i0, v - j0, w - math.floor(w)
        i1, j1, k1 = min(i0 + 1, W - 1), min(j0 + 1, H - 1), (k0 + 1) % K
        c = np.empty((2, 2, 2))
        for a, kk in enumerate((k0, k1)):
            for b, jj in enumerate((j0, j1)):
                for e, ii in enumerate((i0, i1)):
                    c[a, b, e] = grid[kk, jj, ii]
        # value: lerp over u, then v, then w
        cu = c[:, :, 0] * (1 - fu) + c[:, :, 1] * fu          # [w][v]
        cuv = cu[:, 0] * (1 - fv) + cu[:, 1] * fv              # [w]
        val = cuv[0] * (1 - fw) + cuv[1] * fw
        du = c[:, :, 1] - c[:, :, 0]                           # [w][v]
        du_v = du[:, 0] * (1 - fv) + du[:, 1] * fv
        d_u = du_v[0] * (1 - fw) + du_v[1] * fw
        dv = cu[:, 1] - cu[:, 0]
        d_v = dv[0] * (1 - fw) + dv[1] * fw
        d_w = cuv[1] - cuv[0]
        out[n] = (val, d_u / res if inside_u else 0.0, d_v / res if inside_v else 0.0, d_w / dth)
    return out
