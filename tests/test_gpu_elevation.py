"""Elevation-map update on the GPU (scan fusion and nearest-neighbour
inpainting) against the FP64 reference (oracle/elevation.py).

The bar is bit-exact: the per-point arithmetic and the per-cell fold run in
FP64 with the reference's operations in the reference's order (no
contraction), and each cell's float32 height and variance are rounded once at
the end, so every gate decision and every stored value must agree."""
import numpy as np
import pytest

from oracle import elevation as E
from paper_2503_02412_amd import inputs as I
from paper_2503_02412_amd import seb

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _announce(request):
    print(f"\n[gpu-case] {request.node.nodeid}", flush=True)


def small(W, H, res):
    return I.Params(W, H, res, 4, 0.6, 0.4, 6, 4)


def prior_maps(W, H, seed, known_frac=0.5):
    rng = np.random.default_rng(seed)
    h = rng.normal(0.0, 0.3, (H, W)).astype(np.float32)
    v = rng.uniform(1e-4, 4e-3, (H, W)).astype(np.float32)
    h[rng.random((H, W)) > known_frac] = np.nan
    return h, v


def to_ring(a, origin):
    H, W = a.shape
    return np.roll(a, (origin[1] % H, origin[0] % W), axis=(0, 1))


def from_ring(a, origin):
    H, W = a.shape
    return np.roll(a, (-(origin[1] % H), -(origin[0] % W)), axis=(0, 1))


def oracle_fuse(h, v, scan, p, origin):
    cell, z, var = E.process_points(scan["points"], scan["R_B"], scan["p_B"], scan["R_BS"],
                                    scan["p_BS"], scan["Sigma_R"], scan["Sigma_B"],
                                    scan["sigma_range"], scan["sigma_angle"], scan["z_min"],
                                    scan["z_max"], p.resolution, p.width, p.height, *origin)
    return E.fuse(h, v, cell, z, var, scan["mahalanobis"])


def gpu_fuse(fuser, h_ring, v_ring, scan, origin):
    import torch
    n = torch.zeros(1, dtype=torch.int32, device="cuda")
    pts = torch.from_numpy(scan["points"]).cuda()
    fuser.fuse(h_ring, v_ring, origin, pts, scan, n_fused=n)
    torch.cuda.synchronize()
    return int(n.item())


def same(a, b):
    return np.array_equal(np.asarray(a), np.asarray(b), equal_nan=True)


@pytest.mark.parametrize("W,H,res,n_points,origin", [
    (128, 96, 0.1, 30000, (0, 0)),
    (100, 70, 0.05, 20000, (-37, 1234)),       # ring offsets, negative world cells
    (400, 400, 0.05, 200000, (-200, -200)),    # the 400 x 400 @ 0.05 m rolling window
])
def test_fuse_matches_oracle(W, H, res, n_points, origin):
    import torch
    p = small(W, H, res)
    terrain = I.fractal_terrain(W, H, res, seed=W + H, hole_frac=0.05)
    h0, v0 = prior_maps(W, H, seed=W)
    scans = [I.synthetic_scan(terrain, res, n_points, seed=s, origin=origin,
                              max_range=0.45 * min(W, H) * res) for s in (1, 2)]
    with seb.Context(p) as ctx:
        fuser = seb.Fuser(ctx, n_points)
        hr = torch.from_numpy(to_ring(h0, origin)).cuda()
        vr = torch.from_numpy(to_ring(v0, origin)).cuda()
        h, v = h0, v0
        for scan in scans:                        # two scans in a row: the state carries over
            h, v, used = oracle_fuse(h, v, scan, p, origin)
            n = gpu_fuse(fuser, hr, vr, scan, origin)
            gh = from_ring(hr.cpu().numpy(), origin)
            gv = from_ring(vr.cpu().numpy(), origin)
            assert n == used
            assert same(gh, h), np.argwhere(~((gh == h) | (np.isnan(gh) & np.isnan(h))))[:5]
            assert same(gv, v)
        fuser.close()
    assert used > n_points // 4                    # the scan did land on the map


def test_fuse_crowded_cell_and_edges():
    """Crowded cells (folded by a workgroup from LDS), 3000 points in one cell
    (beyond what a workgroup ranks in LDS: sorted in place), an empty scan, and
    a scan whose points all miss the window."""
    import torch
    W, H, res = 64, 48, 0.1
    p = small(W, H, res)
    terrain = np.zeros((H, W), np.float32)
    scan = I.synthetic_scan(terrain, res, 6000, seed=4, max_range=0.35)
    h0, v0 = prior_maps(W, H, seed=5)
    with seb.Context(p) as ctx:
        fuser = seb.Fuser(ctx, 6000)
        hr = torch.from_numpy(h0.copy()).cuda()
        vr = torch.from_numpy(v0.copy()).cuda()
        h, v, used = oracle_fuse(h0, v0, scan, p, (0, 0))
        assert gpu_fuse(fuser, hr, vr, scan, (0, 0)) == used
        assert same(hr.cpu().numpy(), h) and same(vr.cpu().numpy(), v)
        empty = dict(scan, points=scan["points"][:0])
        assert gpu_fuse(fuser, hr, vr, empty, (0, 0)) == 0
        assert same(hr.cpu().numpy(), h)
        assert gpu_fuse(fuser, hr, vr, scan, (10_000, 0)) == 0   # window far away
        assert same(hr.cpu().numpy(), h) and same(vr.cpu().numpy(), v)
        # 3000 returns within one cell: more than a workgroup ranks in LDS
        rng = np.random.default_rng(6)
        one = scan["points"][:1] + rng.normal(0.0, 1e-3, (3000, 3)).astype(np.float32)
        one_scan = dict(scan, points=one.astype(np.float32))
        h, v, used = oracle_fuse(h, v, one_scan, p, (0, 0))
        assert gpu_fuse(fuser, hr, vr, one_scan, (0, 0)) == used
        assert same(hr.cpu().numpy(), h) and same(vr.cpu().numpy(), v)
        fuser.close()
    counts = np.bincount(E.process_points(scan["points"], scan["R_B"], scan["p_B"], scan["R_BS"],
                                          scan["p_BS"], scan["Sigma_R"], scan["Sigma_B"], 0.02,
                                          0.002, -3, 2, res, W, H, 0, 0)[0] + 1)
    assert counts[1:].max() > 8                    # some cells took the workgroup path


def test_fuse_rejects_bad_arguments():
    import torch
    W, H = 32, 32
    p = small(W, H, 0.1)
    scan = I.synthetic_scan(np.zeros((H, W), np.float32), 0.1, 100, seed=1, max_range=1.0)
    pts = torch.from_numpy(scan["points"]).cuda()
    h = torch.zeros((H, W), device="cuda")
    with seb.Context(p) as ctx:
        fuser = seb.Fuser(ctx, 50)
        with pytest.raises(seb.SebError):
            fuser.fuse(h, h.clone(), (0, 0), pts, scan)              # more points than max_points
        fuser.close()
        fuser = seb.Fuser(ctx, 1000)
        for bad in ({"sigma_range": 0.0}, {"mahalanobis": 0.0}, {"z_min": 3.0},
                    {"R_B": np.full(9, np.nan)}):
            with pytest.raises(seb.SebError):
                fuser.fuse(h, h.clone(), (0, 0), pts, dict(scan, **bad))
        fuser.close()
        with pytest.raises(seb.SebError):
            fuser.fuse(h, h, (0, 0), pts, scan)                      # height is variance
        with pytest.raises(seb.SebError):
            seb.Fuser(ctx, 0)


@pytest.mark.parametrize("W,H,radius,ring,hole_frac", [
    (96, 80, 5, (0, 0), 0.3),
    (70, 45, 16, (13, 44), 0.6),
    (33, 20, 0, (2, 3), 0.2),
    (800, 800, 8, (123, 456), 0.15),           # the 800 x 800 map with 15% holes
])
def test_inpaint_matches_oracle(W, H, radius, ring, hole_frac):
    import torch
    p = small(W, H, 0.05)
    h = I.fractal_terrain(W, H, 0.05, seed=W, hole_frac=hole_frac)
    h[0, 0] = np.inf
    want = E.inpaint_nearest(h, radius)
    with seb.Context(p) as ctx:
        src = torch.from_numpy(np.roll(h, (ring[1], ring[0]), axis=(0, 1)).copy()).cuda()
        got = ctx.inpaint(src, radius, ring=ring)
        torch.cuda.synchronize()
        got = np.roll(got.cpu().numpy(), (-ring[1], -ring[0]), axis=(0, 1))
        with pytest.raises(seb.SebError):
            ctx.inpaint(src, 17)
        with pytest.raises(seb.SebError):
            ctx.inpaint(src, 3, out=src)
    assert same(got, want)
    assert np.isfinite(got).mean() >= np.isfinite(h).mean()


def stale_map(terrain, seed, frac=0.05, lift=1.5):
    """The terrain with a fraction of cells standing `lift` metres too high
    (obstacles that have moved away), as the ray casting is meant to clear."""
    rng = np.random.default_rng(seed)
    h = terrain.copy()
    h[rng.random(h.shape) < frac] += lift
    return h


@pytest.mark.parametrize("W,H,res,origin,n_points,margin,robot", [
    (128, 96, 0.1, (0, 0), 20000, 0.0, None),
    (100, 70, 0.05, (-37, 1234), 20000, 0.05, None),
    (400, 400, 0.05, (-200, -200), 30000, 0.0, None),   # the 400 x 400 @ 0.05 m window
    (60, 50, 0.1, (10, -20), 5000, 0.0, (-0.5, -3.2)),  # the sensor outside the window
])
def test_raycast_matches_oracle(W, H, res, origin, n_points, margin, robot):
    import torch
    p = small(W, H, res)
    if robot is None:
        terrain = I.fractal_terrain(W, H, res, seed=W, hole_frac=0.05)
        scan = I.synthetic_scan(terrain, res, n_points, seed=W, origin=origin,
                                max_range=0.6 * min(W, H) * res)
        hm = stale_map(terrain, W)
    else:
        big = I.fractal_terrain(200, 200, res, seed=50, hole_frac=0.05)   # world cells [-100, 100)
        scan = I.synthetic_scan(big, res, n_points, seed=2, origin=(-100, -100), robot_xy=robot,
                                max_range=9.0)
        hm = stale_map(big[origin[1] + 100:origin[1] + 100 + H, origin[0] + 100:origin[0] + 100 + W],
                       7, frac=0.1)
    want, n_want = E.raycast_reset(hm, scan["points"], scan["R_B"], scan["p_B"], scan["R_BS"],
                                   scan["p_BS"], res, origin[0], origin[1], margin)
    with seb.Context(p) as ctx:
        hr = torch.from_numpy(to_ring(hm, origin)).cuda()
        n = torch.zeros(1, dtype=torch.int32, device="cuda")
        ctx.raycast_reset(hr, origin, torch.from_numpy(scan["points"]).cuda(), scan, margin,
                          n_reset=n)
        torch.cuda.synchronize()
        got = from_ring(hr.cpu().numpy(), origin)
        assert int(n.item()) == n_want
        with pytest.raises(seb.SebError):
            ctx.raycast_reset(hr, origin, torch.from_numpy(scan["points"]).cuda(), scan, -1.0)
        # without a count the resets are plain stores: the same map
        hr2 = torch.from_numpy(to_ring(hm, origin)).cuda()
        ctx.raycast_reset(hr2, origin, torch.from_numpy(scan["points"]).cuda(), scan, margin)
        torch.cuda.synchronize()
        assert same(from_ring(hr2.cpu().numpy(), origin), want)
    assert same(got, want)
    assert n_want > 20                               # the rays did clear stale cells
