"""FP64 reference of the elevation-map update that feeds the assessment --
TEST INFRASTRUCTURE.

Only the test-suite, the smoke check and the CPU-baseline leg of the benchmark
may import this module.  It shares no code with the library.

What it computes (Sec. V-A of the paper):
  - each LiDAR point is taken from the sensor frame to the body frame and to
    the map frame, dropped if it lies outside the map or outside a height band
    of the body frame, and given the variance of its height from Eq. 5-9:
        z_l = b3^T (R_B (R_BS p_S + p_BS) + p_B)
        J_S = (R_B R_BS)^T b3,  J_R = (R_BS p_S + p_BS)^ R_B^T b3,  J_B = -b3
        var = J_S^T Sigma_S J_S + J_R^T Sigma_R J_R + J_B^T Sigma_B J_B;
  - the points falling into one map cell update that cell's height and
    variance with a one-dimensional Kalman filter, with the classical
    elevation map's Mahalanobis test for several heights in one cell;
  - cells standing higher than a ray that passes through them are reset to
    unknown (ray casting);
  - unknown cells are filled from the nearest known cell (nearest-neighbour
    inpainting, the method of the experiments).

Readings (the paper leaves these open; the library uses the same ones):
  - frames: the map frame has rotation I (Sec. V-A); world cell (gx, gy) =
    (floor(x / res), floor(y / res)) covers [gx res, (gx+1) res) x ...; a
    window whose logical cell (0, 0) is world cell (ox, oy) holds logical
    cells [0, W) x [0, H), stored at ring position (gx mod W, gy mod H);
  - height: the map height of a point is its map-frame z (b3^T p_l with +p_B;
    the printed -p_B only flips J_B's sign, which the variance does not see);
  - height band: q_z (body-frame z of the point) in [z_min, z_max];
  - Sigma_R: covariance of a body-frame rotation perturbation R_B Exp(d),
    the convention under which the printed J_R is the derivative;
  - sensor model: Sigma_S = s_r^2 u u^T + (s_a r)^2 (I - u u^T), u = p_S / r,
    r = |p_S|: range noise along the beam, angular noise across it; written
    without square roots as
        J_S^T Sigma_S J_S = s_r^2 (J_S.p)^2 / r^2 + s_a^2 (r^2 - (J_S.p)^2);
  - fusion order: the points of a cell in increasing point index; a point
    with (z - h)^2 > tau^2 v (Mahalanobis distance above tau) replaces the
    cell if it is higher and is dropped if it is lower; otherwise
        h <- (v z + s h) / (v + s),  v <- v s / (v + s);
    an unknown cell (non-finite height) takes the point as it is.  The fold
    runs in FP64 and the cell's float32 height and variance are written at
    the end;
  - ray casting: before the points are fused, each finite point's segment
    from the sensor (R_B p_BS + p_B) resets the known cells it crosses --
    cells its xy projection passes through with a parameter interval
    t0 < t1 by slab clipping, other than the point's own cell -- whose height
    exceeds max(z(t0), z(t1)) + margin; decisions use the heights before the
    scan, so the result is a union and does not depend on ray order;
  - inpainting: an unknown cell takes the height of the known cell with the
    smallest (dx^2 + dy^2, dy, dx) within the radius (dx, dy signed, ring
    order irrelevant: logical coordinates); none within it: stays unknown,
    written as NaN (also where it was +-Inf).

Arithmetic is written out scalar by scalar (no matrix products) so that every
IEEE operation, and so every floor and comparison, is the one the kernels
perform.
"""
from __future__ import annotations

import math

import numpy as np


def _mat(m) -> np.ndarray:
    return np.asarray(m, dtype=np.float64).reshape(3, 3)


def _vec(v) -> np.ndarray:
    return np.asarray(v, dtype=np.float64).reshape(3)


def process_points(points, R_B, p_B, R_BS, p_BS, Sigma_R, Sigma_B, s_r, s_a,
                   z_min, z_max, res, W, H, origin_x, origin_y):
    """Per point: (logical cell index ly * W + lx, or -1 if dropped), map-frame
    height, height variance; all points [n][3] in the sensor frame."""
    P = np.asarray(points, dtype=np.float64).reshape(-1, 3)
    px, py, pz = P[:, 0], P[:, 1], P[:, 2]
    A, a = _mat(R_BS), _vec(p_BS)
    R, b = _mat(R_B), _vec(p_B)
    SR, SB = _mat(Sigma_R), _mat(Sigma_B)
    # body frame: q = R_BS p + p_BS
    q0 = A[0, 0] * px + A[0, 1] * py + A[0, 2] * pz + a[0]
    q1 = A[1, 0] * px + A[1, 1] * py + A[1, 2] * pz + a[1]
    q2 = A[2, 0] * px + A[2, 1] * py + A[2, 2] * pz + a[2]
    # map frame: l = R_B q + p_B
    lx = R[0, 0] * q0 + R[0, 1] * q1 + R[0, 2] * q2 + b[0]
    ly = R[1, 0] * q0 + R[1, 1] * q1 + R[1, 2] * q2 + b[1]
    lz = R[2, 0] * q0 + R[2, 1] * q1 + R[2, 2] * q2 + b[2]
    # J_S = (R_B R_BS)^T b3: row 2 of R_B R_BS
    j0 = R[2, 0] * A[0, 0] + R[2, 1] * A[1, 0] + R[2, 2] * A[2, 0]
    j1 = R[2, 0] * A[0, 1] + R[2, 1] * A[1, 1] + R[2, 2] * A[2, 1]
    j2 = R[2, 0] * A[0, 2] + R[2, 1] * A[1, 2] + R[2, 2] * A[2, 2]
    jp = j0 * px + j1 * py + j2 * pz
    r2 = px * px + py * py + pz * pz
    with np.errstate(divide="ignore", invalid="ignore"):
        sensor = np.where(r2 > 0.0, s_r * s_r * (jp * jp) / r2 + s_a * s_a * (r2 - jp * jp),
                          s_r * s_r)
    # J_R = q x g with g = R_B^T b3 = row 2 of R_B
    g0, g1, g2 = R[2, 0], R[2, 1], R[2, 2]
    k0 = q1 * g2 - q2 * g1
    k1 = q2 * g0 - q0 * g2
    k2 = q0 * g1 - q1 * g0
    rot = (k0 * (SR[0, 0] * k0 + SR[0, 1] * k1 + SR[0, 2] * k2)
           + k1 * (SR[1, 0] * k0 + SR[1, 1] * k1 + SR[1, 2] * k2)
           + k2 * (SR[2, 0] * k0 + SR[2, 1] * k1 + SR[2, 2] * k2))
    var = sensor + rot + SB[2, 2]
    gx = np.floor(lx / res)
    gy = np.floor(ly / res)
    cx = gx - origin_x
    cy = gy - origin_y
    keep = (q2 >= z_min) & (q2 <= z_max) & (cx >= 0) & (cx < W) & (cy >= 0) & (cy < H)
    keep &= np.isfinite(lz)
    cell = np.where(keep, cy * W + cx, -1).astype(np.int64)
    return cell, lz, var


def fuse(height: np.ndarray, variance: np.ndarray, cell, z, var, tau: float):
    """Fold the points into the logical [H][W] float32 maps; returns the new
    (height, variance) float32 maps and the number of points that changed a
    cell (fused, or replaced it)."""
    Hm = np.asarray(height, dtype=np.float32)
    Vm = np.asarray(variance, dtype=np.float32)
    W = Hm.shape[1]
    state: dict[int, list[float]] = {}
    used = 0
    tau2 = float(tau) * float(tau)
    for i in np.argsort(np.where(np.asarray(cell) < 0, np.iinfo(np.int64).max, cell),
                        kind="stable"):
        c = int(cell[i])
        if c < 0:
            break
        if c not in state:
            state[c] = [float(Hm.flat[c]), float(Vm.flat[c])]
        h, v = state[c]
        zi, si = float(z[i]), float(var[i])
        if not math.isfinite(h):
            h, v = zi, si
            used += 1
        else:
            dz = zi - h
            if dz * dz > tau2 * v:
                if zi > h:
                    h, v = zi, si
                    used += 1
            else:
                h = (v * zi + si * h) / (v + si)
                v = (v * si) / (v + si)
                used += 1
        state[c] = [h, v]
    Ho, Vo = Hm.copy(), Vm.copy()
    for c, (h, v) in state.items():
        Ho.flat[c] = np.float32(h)
        Vo.flat[c] = np.float32(v)
    del W
    return Ho, Vo, used


def inpaint_nearest(height: np.ndarray, radius: int) -> np.ndarray:
    """Nearest-neighbour fill of the non-finite cells of a logical [H][W] map
    (brute force over every known cell within the radius)."""
    Hm = np.asarray(height, dtype=np.float32)
    out = Hm.copy()
    known = np.isfinite(Hm)
    Hn, Wn = Hm.shape
    r2max = radius * radius
    for y, x in zip(*np.nonzero(~known)):
        out[y, x] = np.nan               # a cell left unknown reads NaN
        # every known cell within the radius lies in this box
        y0, y1 = max(0, y - radius), min(Hn, y + radius + 1)
        x0, x1 = max(0, x - radius), min(Wn, x + radius + 1)
        ky, kx = np.nonzero(known[y0:y1, x0:x1])
        dy = ky + y0 - y
        dx = kx + x0 - x
        d2 = dx * dx + dy * dy
        sel = d2 <= r2max
        if not sel.any():
            continue
        order = np.lexsort((dx[sel], dy[sel], d2[sel]))
        out[y, x] = Hm[y0 + ky[sel][order[0]], x0 + kx[sel][order[0]]]
    return out


def sensor_origin(R_B, p_B, p_BS):
    """Map-frame position of the sensor: R_B p_BS + p_B."""
    R, b, a = _mat(R_B), _vec(p_B), _vec(p_BS)
    return (R[0, 0] * a[0] + R[0, 1] * a[1] + R[0, 2] * a[2] + b[0],
            R[1, 0] * a[0] + R[1, 1] * a[1] + R[1, 2] * a[2] + b[1],
            R[2, 0] * a[0] + R[2, 1] * a[1] + R[2, 2] * a[2] + b[2])


def map_points(points, R_B, p_B, R_BS, p_BS):
    """Map-frame coordinates of sensor-frame points (the same operations as
    process_points)."""
    P = np.asarray(points, dtype=np.float64).reshape(-1, 3)
    px, py, pz = P[:, 0], P[:, 1], P[:, 2]
    A, a = _mat(R_BS), _vec(p_BS)
    R, b = _mat(R_B), _vec(p_B)
    q0 = A[0, 0] * px + A[0, 1] * py + A[0, 2] * pz + a[0]
    q1 = A[1, 0] * px + A[1, 1] * py + A[1, 2] * pz + a[1]
    q2 = A[2, 0] * px + A[2, 1] * py + A[2, 2] * pz + a[2]
    lx = R[0, 0] * q0 + R[0, 1] * q1 + R[0, 2] * q2 + b[0]
    ly = R[1, 0] * q0 + R[1, 1] * q1 + R[1, 2] * q2 + b[1]
    lz = R[2, 0] * q0 + R[2, 1] * q1 + R[2, 2] * q2 + b[2]
    return lx, ly, lz


def _slab(c, res, s, d):
    """Parameter interval [lo, hi] of s + t d inside [c res, (c + 1) res) along
    one axis (d == 0: everything or nothing)."""
    c = np.asarray(c, dtype=np.float64)
    lo_edge, hi_edge = c * res, (c + 1.0) * res
    if d != 0.0:
        t1 = (lo_edge - s) / d
        t2 = (hi_edge - s) / d
        return np.minimum(t1, t2), np.maximum(t1, t2)
    inside = (lo_edge <= s) & (s < hi_edge)
    return np.where(inside, -np.inf, np.inf), np.where(inside, np.inf, -np.inf)


def raycast_reset(height, points, R_B, p_B, R_BS, p_BS, res, origin_x, origin_y, margin):
    """Ray-casting reset (Sec. V-A): a known cell crossed by the segment from
    the sensor to a point (its projection passing through the cell's
    interior), other than the point's own cell, becomes unknown if its height
    exceeds the segment's highest z over the crossing by more than `margin`.
    Decided against the heights before the scan; returns (new map, number of
    cells reset).  Brute force over each ray's bounding box of cells."""
    Hm = np.asarray(height, dtype=np.float32)
    Hn, Wn = Hm.shape
    sx, sy, sz = sensor_origin(R_B, p_B, p_BS)
    lx, ly, lz = map_points(points, R_B, p_B, R_BS, p_BS)
    reset = np.zeros(Hm.shape, dtype=bool)
    si, sj = math.floor(sx / res), math.floor(sy / res)
    for ex, ey, ez in zip(lx, ly, lz):
        if not (math.isfinite(ex) and math.isfinite(ey) and math.isfinite(ez)):
            continue
        ei, ej = math.floor(ex / res), math.floor(ey / res)
        i0, i1 = max(min(si, ei), origin_x), min(max(si, ei), origin_x + Wn - 1)
        j0, j1 = max(min(sj, ej), origin_y), min(max(sj, ej), origin_y + Hn - 1)
        if i0 > i1 or j0 > j1:
            continue
        jj, ii = np.mgrid[j0:j1 + 1, i0:i1 + 1]
        dx, dy, dz = ex - sx, ey - sy, ez - sz
        xlo, xhi = _slab(ii, res, sx, dx)
        ylo, yhi = _slab(jj, res, sy, dy)
        t0 = np.maximum(np.maximum(xlo, ylo), 0.0)
        t1 = np.minimum(np.minimum(xhi, yhi), 1.0)
        crossed = (t1 > t0) & ~((ii == ei) & (jj == ej))
        zmax = np.maximum(sz + t0 * dz, sz + t1 * dz)
        h = Hm[jj - origin_y, ii - origin_x].astype(np.float64)
        with np.errstate(invalid="ignore"):
            hit = crossed & (h > zmax + margin)
        reset[jj[hit] - origin_y, ii[hit] - origin_x] = True
    out = Hm.copy()
    out[reset] = np.nan
    return out, int(reset.sum())
