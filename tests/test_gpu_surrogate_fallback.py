"""The surrogate's fallback on the flags a trained network really produces:
scattered states (predicted risk near risk_max, windows with too few known
cells, cells without a reference height), so the compacted 64-state items are
sparse and their bounding boxes unaligned.  Every state the network does not
answer must equal the plain kernel (up to the fallback's summation order) and
meet the oracle parity rule (Sec. V-B, Alg. 1); every state it answers must
carry the surrogate bit.  Also counts the unsafe direction: states the network
calls traversable where Alg. 1 finds an explicit obstacle."""
import numpy as np
import pytest

from paper_2503_02412_amd import inputs as I
from paper_2503_02412_amd import seb
from paper_2503_02412_amd.surrogate import TrainingData, train
from parity import compare, to_numpy

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _announce(request):
    print(f"\n[gpu-case] {request.node.nodeid}", flush=True)


@pytest.fixture(scope="module")
def trained_net():
    data = TrainingData(count=600_000)
    net = seb.Net(seed=3, max_batch=4096)
    hist = train(net, data, steps=500, batch=4096)
    assert hist[-20:].mean() < 0.5 * hist[:20].mean()
    return net


def _case(footprint, precision):
    if footprint == "standard":
        return I.CONFIG2.with_(precision=precision), I.config2_map(I.SURROGATE_EVAL_SEEDS[0])
    # 2.0 x 1.2 m on 40 x 24 samples, on a ragged crop of another evaluation map
    p = I.CONFIG2.with_(width=120, height=104, fp_length=2.0, fp_width=1.2, fp_nl=40, fp_nw=24,
                        precision=precision)
    return p, I.config2_map(I.SURROGATE_EVAL_SEEDS[1])[40:144, 30:150].copy()


@pytest.mark.parametrize("footprint", ["standard", "large"])
@pytest.mark.parametrize("precision", [0, 1])
def test_sparse_fallback_matches_plain_and_oracle(orc, trained_net, footprint, precision):
    import torch
    p, h = _case(footprint, precision)
    with seb.Context(p) as ctx:
        sur = seb.Surrogate(ctx)
        dh = torch.from_numpy(h).cuda()
        nf = torch.zeros(1, dtype=torch.int32, device="cuda")
        a = to_numpy(sur.infer(trained_net, dh, band=0.1, min_known=0.5, n_fallback=nf))
        b = to_numpy(ctx.assess(dh))
        torch.cuda.synchronize()
        n_fb = int(nf.item())
    fb = (a["status"] & seb.ST_SURROGATE) == 0
    print(footprint, precision, "fallback", fb.mean())
    assert n_fb == int(fb.sum())
    assert 0.01 < fb.mean() < 0.5
    # answered states: valid, surrogate, nothing else but the traversable bit
    ans = a["status"][~fb]
    assert np.all((ans & ~np.uint8(seb.ST_TRAV)) == seb.ST_VALID | seb.ST_SURROGATE)
    # the flags are scattered: most 16 x 4 blocks that hold a fallback state
    # hold answered states too
    K, H, W = fb.shape
    Hb, Wb = H // 4 * 4, W // 16 * 16
    blk = fb[:, :Hb, :Wb].reshape(K, Hb // 4, 4, Wb // 16, 16).sum(axis=(2, 4))
    n_partial = np.count_nonzero((blk > 0) & (blk < 64))
    print("blocks with fallback states", np.count_nonzero(blk), "partly answered", n_partial)
    assert n_partial >= 50
    # fallback states against the plain kernel
    assert np.array_equal(a["status"][fb] & 9, b["status"][fb] & 9)
    v = fb & ((b["status"] & 1) > 0)
    for f in ("z", "roll", "pitch", "risk"):
        assert np.array_equal(np.isnan(a[f][fb]), np.isnan(b[f][fb])), f
        d = np.abs(a[f][v].astype(np.float64) - b[f][v])
        print(f, d.max(initial=0.0))
        assert d.max(initial=0.0) <= 2e-5, f
    # and against the oracle, state by state
    k, y, x = np.nonzero(fb)
    o = orc.assess_list(p, h, x, y, k)
    print(compare({f: a[f][fb] for f in ("z", "roll", "pitch", "risk", "status")}, o, p))


def test_unsafe_direction_is_counted_and_small(orc, trained_net):
    """States answered as traversable where the oracle sets a curvature or
    tilt obstacle bit: counted, and kept small (a network trained 500 steps);
    the SDF counts every non-traversable answer as an obstacle."""
    import torch
    p, h = _case("standard", 0)
    with seb.Context(p) as ctx:
        sur = seb.Surrogate(ctx)
        a = to_numpy(sur.infer(trained_net, torch.from_numpy(h).cuda(), band=0.1,
                               min_known=0.5))
        sdf = ctx.sdf(torch.from_numpy(a["status"]).cuda(), 4, True).cpu().numpy()
    o = orc.assess_rect(p, h)
    ans = (a["status"] & seb.ST_SURROGATE) > 0
    unsafe = ans & ((a["status"] & seb.ST_TRAV) > 0) & ((o.status & 6) > 0)
    print("answered", ans.sum(), "unsafe", unsafe.sum(), unsafe.sum() / max(1, ans.sum()))
    assert unsafe.sum() <= 0.01 * ans.sum()
    # non-traversable answers are obstacles of the SDF, traversable ones free
    nt = ans & ((a["status"] & seb.ST_TRAV) == 0)
    assert nt.any()
    assert np.all(sdf[nt] < 0)
    assert np.all(sdf[ans & ~nt] > 0)
