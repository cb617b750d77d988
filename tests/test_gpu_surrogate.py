"""GPU surrogate network: forward and gradients against the FP64 reference,
training, checkpoints."""
import numpy as np
import pytest

from oracle import surrogate as S
from paper_2503_02412_amd import inputs as I
from paper_2503_02412_amd import seb

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _announce(request):
    print(f"\n[gpu-case] {request.node.nodeid}", flush=True)


def ref_params(vec):
    """Reference parameters as the GPU sees them: GEMM weights rounded to bf16."""
    P = S.unflatten(vec.astype(np.float64))
    for k in ("W1", "W2", "W3", "W4", "W5"):
        P[k] = S.bf16_round(P[k])
    return P


def random_setup(n_maps=3, size=40, B=64, seed=0):
    import torch
    rng = np.random.default_rng(seed)
    maps = np.stack([I.surrogate_training_map(7000 + i, size) for i in range(n_maps)])
    K = 12
    known = np.argwhere(np.isfinite(maps))            # (map, y, x) of known cells
    # holes whose z target is relative to the mean of their known neighbours
    holes = np.array([c for c in np.argwhere(~np.isfinite(maps))
                      if S.reference_height(maps[c[0]], c[1], c[2]) is not None])
    assert len(holes) >= 8
    pick = np.concatenate([known[rng.integers(0, len(known), B - 8)],
                           holes[rng.integers(0, len(holes), 8)]])
    samp = np.c_[pick, rng.integers(0, K, B)].astype(np.int32)
    labels = {k: rng.normal(0, 0.3, (n_maps, K, size, size)).astype(np.float32)
              for k in ("z", "roll", "pitch", "risk")}
    dev = {k: torch.from_numpy(v).cuda() for k, v in labels.items()}
    return maps, samp, labels, K, torch.from_numpy(maps).cuda(), torch.from_numpy(samp).cuda(), dev


def ref_inputs(maps, samp, K, res=0.1):
    X = np.stack([S.encode(maps[m], res, cy, cx) for m, cy, cx, _ in samp])
    th = 2 * np.pi * samp[:, 3] / K
    sc = np.stack([np.sin(th), np.cos(th)], 1).astype(np.float32).astype(np.float64)
    return S.bf16_round(X.astype(np.float32)), sc


def test_forward_matches_reference():
    import torch
    net = seb.Net(seed=3, max_batch=256)
    rng = np.random.default_rng(1)
    vec = (rng.normal(0, 0.15, S.N_PARAMS)).astype(np.float32)
    net.set_params(vec)
    maps, samp, _, K, dmaps, dsamp, _ = random_setup(B=64)
    y = net.forward(dmaps, dsamp, 0.1, K).cpu().numpy().astype(np.float64)
    X, sc = ref_inputs(maps, samp, K)
    yr, _ = S.forward(ref_params(vec), X, sc)
    err = np.abs(y - yr).max() / (np.abs(yr).max() + 1e-12)
    print("forward rel err", err)
    assert err < 3e-2


def test_gradients_match_reference():
    import torch
    net = seb.Net(seed=4, max_batch=256)
    rng = np.random.default_rng(2)
    vec = (rng.normal(0, 0.15, S.N_PARAMS)).astype(np.float32)
    net.set_params(vec)
    maps, samp, labels, K, dmaps, dsamp, dlab = random_setup(B=96, seed=5)
    grad = torch.zeros(S.N_PARAMS, dtype=torch.float32, device="cuda")
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    net.train_step(dmaps, dlab, dsamp, 0.1, K, 1e-3, loss=loss, grad=grad)
    g = grad.cpu().numpy().astype(np.float64)
    X, sc = ref_inputs(maps, samp, K)
    P = ref_params(vec)
    t = np.stack([S.targets(maps[m], labels["z"][m, k, cy, cx], labels["roll"][m, k, cy, cx],
                            labels["pitch"][m, k, cy, cx], labels["risk"][m, k, cy, cx], cy, cx)
                  for m, cy, cx, k in samp])
    # Exact FP64 gradients, and FP64 gradients with activations and deltas
    # rounded to bf16 where the kernels store them.
    y, cache = S.forward(P, X, sc)
    L, dy = S.loss(y, t)
    gr = S.flatten(S.backward(P, cache, dy))
    yb, cb = S.forward(P, X, sc, rnd=S.bf16_round)
    Lb, dyb = S.loss(yb, t)
    gb = S.flatten(S.backward(P, cb, dyb, rnd=S.bf16_round))
    assert abs(float(loss.item()) - Lb) / Lb < 1e-3
    assert abs(float(loss.item()) - L) / L < 3e-2
    o = 0
    for name, shape in S.SHAPES:
        n = int(np.prod(shape))
        a = g[o:o + n]
        rel_b = np.linalg.norm(a - gb[o:o + n]) / (np.linalg.norm(gb[o:o + n]) + 1e-30)
        rel = np.linalg.norm(a - gr[o:o + n]) / (np.linalg.norm(gr[o:o + n]) + 1e-30)
        print(f"{name}: vs bf16-rounded FP64 {rel_b:.2e}, vs exact FP64 {rel:.2e}")
        assert rel_b < 1e-2, name
        assert rel < 0.15, name
        o += n
    # the weights did not move
    assert np.array_equal(net.params(), vec)


def test_training_step_decreases_loss_and_checkpoints(tmp_path):
    import torch
    maps, samp, labels, K, dmaps, dsamp, dlab = random_setup(B=256, seed=9)
    net = seb.Net(seed=11, max_batch=256)
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    hist = []
    for step in range(60):
        net.train_step(dmaps, dlab, dsamp, 0.1, K, 3e-3, loss=loss)
        hist.append(float(loss.item()))
    assert hist[-1] < 0.7 * hist[0], hist[::10]
    path = str(tmp_path / "net.bin")
    net.save(path)
    other = seb.Net(seed=12, max_batch=256)
    other.load(path)
    assert np.array_equal(other.params(), net.params())
    y0 = net.forward(dmaps, dsamp, 0.1, K)
    y1 = other.forward(dmaps, dsamp, 0.1, K)
    assert torch.equal(y0, y1)
    with open(path, "r+b") as f:
        f.write(b"XXXX")
    with pytest.raises(seb.SebError):
        other.load(path)
