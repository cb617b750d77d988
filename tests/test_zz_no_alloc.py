"""seb_fuse_scan_static (no allocation, static device workspace) against
seb_fuse_scan with a fuser: the same kernels, so the results must agree bit
for bit, on two calls in a row (the second on a smaller map and scan, so
stale workspace contents from the first call would show), plus the size
limits it rejects before launching anything."""
import numpy as np
import pytest

from paper_2503_02412_amd import inputs as I
from paper_2503_02412_amd import seb

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _announce(request):
    print(f"\n[gpu-case] {request.node.nodeid}", flush=True)


def small(W, H, res):
    return I.Params(W, H, res, 4, 0.6, 0.4, 6, 4)


def prior_maps(W, H, seed):
    rng = np.random.default_rng(seed)
    h = rng.normal(0.0, 0.3, (H, W)).astype(np.float32)
    v = rng.uniform(1e-4, 4e-3, (H, W)).astype(np.float32)
    h[rng.random((H, W)) > 0.5] = np.nan
    return h, v


def run_pair(W, H, res, n_points, origin, seed):
    import torch
    p = small(W, H, res)
    terrain = I.fractal_terrain(W, H, res, seed=seed, hole_frac=0.05)
    scan = I.synthetic_scan(terrain, res, n_points, seed=seed, origin=origin,
                            max_range=0.45 * min(W, H) * res)
    h0, v0 = prior_maps(W, H, seed)
    pts = torch.from_numpy(scan["points"]).cuda()
    with seb.Context(p) as ctx:
        fuser = seb.Fuser(ctx, n_points)
        ha, va = torch.from_numpy(h0).cuda(), torch.from_numpy(v0).cuda()
        hb, vb = ha.clone(), va.clone()
        na = torch.zeros(1, dtype=torch.int32, device="cuda")
        nb = torch.zeros(1, dtype=torch.int32, device="cuda")
        fuser.fuse(ha, va, origin, pts, scan, n_fused=na)
        seb.fuse_scan_static(ctx, hb, vb, origin, pts, scan, n_fused=nb)
        torch.cuda.synchronize()
        fuser.close()
        same = lambda a, b: np.array_equal(a.cpu().numpy(), b.cpu().numpy(), equal_nan=True)
        assert int(na.item()) == int(nb.item()) > n_points // 4
        assert same(ha, hb) and same(va, vb)


def test_static_fuse_equals_fuser_twice():
    run_pair(400, 400, 0.05, 200_000, (-200, -200), seed=3)
    run_pair(96, 64, 0.1, 20_000, (17, -5), seed=4)       # smaller map and scan


def test_static_fuse_rejects_oversize():
    import torch
    p = small(600, 500, 0.05)                              # 300,000 cells > 2^18
    with seb.Context(p) as ctx:
        h = torch.zeros((500, 600), dtype=torch.float32, device="cuda")
        v = torch.ones_like(h)
        pts = torch.zeros((10, 3), dtype=torch.float32, device="cuda")
        scan = I.synthetic_scan(np.zeros((8, 8), np.float32), 0.05, 10, seed=1)
        with pytest.raises(seb.SebError):
            seb.fuse_scan_static(ctx, h, v, (0, 0), pts, scan)
    p = small(64, 64, 0.1)
    with seb.Context(p) as ctx:
        h = torch.zeros((64, 64), dtype=torch.float32, device="cuda")
        v = torch.ones_like(h)
        pts = torch.zeros(((1 << 18) + 1, 3), dtype=torch.float32, device="cuda")
        scan = I.synthetic_scan(np.zeros((8, 8), np.float32), 0.1, 10, seed=1)
        with pytest.raises(seb.SebError):
            seb.fuse_scan_static(ctx, h, v, (0, 0), pts, scan)
