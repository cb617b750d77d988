"""Pins of the FP64 surrogate-network reference (oracle/surrogate.py)."""
import numpy as np
import pytest

from oracle import surrogate as S


def small_params(rng, scale=0.3):
    return {n: rng.normal(0, scale, s) for n, s in S.SHAPES}


def test_parameter_count():
    assert S.N_PARAMS == 16 * 48 + 16 + 32 * 144 + 32 + 128 * 800 + 256 + 128 + 64 * 128 + 64 + 256 + 4
    rng = np.random.default_rng(0)
    p = small_params(rng)
    back = S.unflatten(S.flatten(p))
    for n, _ in S.SHAPES:
        assert np.array_equal(back[n], p[n])


def test_conv_stride2_picks_strided_pixels():
    # A delta kernel at tap (i, j) returns the input at (2a + i, 2b + j).
    rng = np.random.default_rng(1)
    X = rng.normal(size=(2, 3, 24, 24))
    for (c, i, j) in [(0, 0, 0), (2, 3, 1), (1, 2, 3)]:
        W = np.zeros((1, 3, 4, 4))
        W[0, c, i, j] = 1.0
        out = S.conv_stride2(X, W)
        assert out.shape == (2, 1, 11, 11)
        for a in range(11):
            for b in range(11):
                assert out[1, 0, a, b] == X[1, c, 2 * a + i, 2 * b + j]


def test_encode_plane_and_holes():
    res = 0.1
    iy, ix = np.mgrid[0:40, 0:40]
    H = (0.02 * ix - 0.05 * iy).astype(np.float32)
    X = S.encode(H, res, 20, 20)
    assert np.allclose(X[0], 0.2, atol=1e-5) and np.allclose(X[1], -0.5, atol=1e-5)
    assert np.all(X[2] == 1.0)
    H2 = H.copy()
    H2[20, 21] = np.nan
    X2 = S.encode(H2, res, 20, 20)
    # pixel (12, 13) is the cell itself: unknown; its left neighbour loses dx
    assert X2[2, 12, 13] == 0 and X2[0, 12, 13] == 0 and X2[1, 12, 13] == 0
    assert X2[0, 12, 12] == 0 and X2[1, 11, 13] == 0
    # near the map edge the out-of-map cells are unknown
    X3 = S.encode(H, res, 2, 37)
    assert X3[2, 0, 0] == 0 and X3[2, 12, 12] == 1 and X3[2, 12, 15] == 0


def test_reference_height():
    """The z target is relative to the own cell, else the mean of the known
    8-neighbours (in-map only), else undefined."""
    H = np.arange(1.0, 10.0).reshape(3, 3).astype(np.float32)
    assert S.reference_height(H, 1, 1) == 5.0
    H[1, 1] = np.nan
    assert S.reference_height(H, 1, 1) == 5.0          # (1+2+3+4+6+7+8+9) / 8
    H[0, 0] = np.inf                                    # +-Inf is unknown too
    assert S.reference_height(H, 1, 1) == 39.0 / 7
    H[0, 2] = 2.0 ** 61                                 # beyond the height limit
    assert S.reference_height(H, 1, 1) == 6.0
    G = np.full((4, 5), np.nan, np.float32)
    G[1, 1], G[0, 1], G[3, 4] = 0.5, 1.5, 9.0
    assert S.reference_height(G, 0, 0) == 1.0           # corner: 3 in-map neighbours
    assert S.reference_height(G, 1, 3) is None and S.reference_height(G, 3, 3) == 9.0
    # a plane: the neighbour mean of a hole is the plane's height there
    iy, ix = np.mgrid[0:9, 0:9]
    P = (0.3 * ix - 0.7 * iy + 2.0).astype(np.float64)
    P[4, 4] = np.nan
    assert abs(S.reference_height(P, 4, 4) - (0.3 * 4 - 0.7 * 4 + 2.0)) < 1e-12
    t = S.targets(P, 1.6, 0.1, -0.2, 0.3, 4, 4)
    assert np.allclose(t, [(1.6 - 0.4) / S.S_Z, 0.1 / S.S_A, -0.2 / S.S_A, 0.3])


def test_gradients_match_finite_differences():
    rng = np.random.default_rng(2)
    P = small_params(rng, 0.2)
    B = 3
    X = rng.normal(0, 1, (B, 3, 24, 24))
    sc = rng.normal(0, 1, (B, 2))
    t = rng.normal(0, 1, (B, 4))
    y, cache = S.forward(P, X, sc)
    L, dy = S.loss(y, t)
    g = S.backward(P, cache, dy)
    eps = 1e-6
    for name, shape in S.SHAPES:
        idx = [tuple(rng.integers(0, s) for s in shape) for _ in range(6)]
        for ii in idx:
            Pp = {k: v.copy() for k, v in P.items()}
            Pm = {k: v.copy() for k, v in P.items()}
            Pp[name][ii] += eps
            Pm[name][ii] -= eps
            Lp = S.loss(S.forward(Pp, X, sc)[0], t)[0]
            Lm = S.loss(S.forward(Pm, X, sc)[0], t)[0]
            fd = (Lp - Lm) / (2 * eps)
            assert abs(fd - g[name][ii]) <= 1e-6 * max(1.0, abs(fd)), (name, ii, fd, g[name][ii])


def test_bf16_round_matches_torch():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(3)
    x = np.concatenate([rng.normal(0, 1, 1000), rng.normal(0, 1e-3, 1000),
                        np.array([1.0 + 2 ** -8, 1.0 + 3 * 2 ** -9, -2.5, 0.0])]).astype(np.float32)
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(S.bf16_round(x), ref)


def test_adam_matches_torch():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(4)
    theta = rng.normal(size=50)
    p = torch.nn.Parameter(torch.tensor(theta.copy()))
    opt = torch.optim.Adam([p], lr=1e-2)
    m = np.zeros_like(theta)
    v = np.zeros_like(theta)
    th = theta.copy()
    for step in range(1, 6):
        g = rng.normal(size=50)
        p.grad = torch.tensor(g.copy())
        opt.step()
        th, m, v = S.adam_step(th, g, m, v, step, 1e-2)
        assert np.allclose(th, p.detach().numpy(), rtol=0, atol=1e-12)


def test_loss_gradient():
    rng = np.random.default_rng(5)
    y = rng.normal(size=(4, 4))
    t = rng.normal(size=(4, 4))
    L, dy = S.loss(y, t)
    eps = 1e-7
    for i in range(4):
        for o in range(4):
            yp = y.copy()
            yp[i, o] += eps
            assert abs((S.loss(yp, t)[0] - L) / eps - dy[i, o]) < 1e-5
