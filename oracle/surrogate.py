"""FP64 reference of the learned surrogate network -- TEST INFRASTRUCTURE.

Only the test-suite may import this module.  It is the plain definition the
HIP forward/backward kernels are checked against; it shares no code with the
library (the parameter file layout below is the one interface both sides
implement, each in its own code).

The surrogate maps the terrain around a cell, plus the yaw (sin, cos), to the
four outputs of the assessment (Sec. III Eq. 1-3 and Sec. V-B Alg. 1): the
plane height z (relative to the cell's own height), roll, pitch and risk.  The
paper mentions learned traversability models and their uncertainty (Sec. II),
which is why the library falls back to the plain method where the network is
out of distribution or near the risk threshold.

Definition (patch form).  For the cell (cy, cx) of a height map H (NaN =
unknown, res metres per cell) the input has three 24 x 24 channels; pixel
(i, j) stands for map cell (y, x) = (cy - 12 + i, cx - 12 + j):
    v(y, x)  = 1 if H(y, x) is inside the map and finite, else 0
    c0[i, j] = v(y, x) v(y, x+1) (H(y, x+1) - H(y, x)) / res
    c1[i, j] = v(y, x) v(y+1, x) (H(y+1, x) - H(y, x)) / res
    c2[i, j] = v(y, x)
Layers (ReLU after every layer but the last):
    conv1  3 -> 16, 4 x 4, stride 2            -> 16 x 11 x 11
    conv2 16 -> 32, 3 x 3, stride 2            -> 32 x 5 x 5
    flatten in (a, b, channel) order           -> 800
    fc1   800 + 2 (sin yaw, cos yaw) -> 128
    fc2   128 -> 64
    fc3    64 -> 4
Outputs y = (dz / S_Z, roll / S_A, pitch / S_A, risk) with S_Z = 0.05 m and
S_A = 0.5 rad, where dz = z - h_ref and h_ref is H(cy, cx) when known, else
the mean of the known in-map cells among its eight neighbours (a reading: the
paper does not say what the height output is relative to; expressing it
against nearby known ground lets the network answer states whose own cell is
a hole).  A state with no such cell has no reference and no network output.

Parameter vector layout (float32, in this order, C order within each array):
    W1 [16,3,4,4]  b1 [16]  W2 [32,16,3,3]  b2 [32]  W3 [128,800]  Wy [128,2]
    b3 [128]  W4 [64,128]  b4 [64]  W5 [4,64]  b5 [4]
"""
from __future__ import annotations

import numpy as np

PATCH = 24
HALF = 12
S_Z = 0.05
S_A = 0.5
SHAPES = [("W1", (16, 3, 4, 4)), ("b1", (16,)), ("W2", (32, 16, 3, 3)), ("b2", (32,)),
          ("W3", (128, 800)), ("Wy", (128, 2)), ("b3", (128,)), ("W4", (64, 128)),
          ("b4", (64,)), ("W5", (4, 64)), ("b5", (4,))]
N_PARAMS = int(sum(np.prod(s) for _, s in SHAPES))


def unflatten(vec: np.ndarray) -> dict:
    out, o = {}, 0
    for name, shape in SHAPES:
        n = int(np.prod(shape))
        out[name] = np.asarray(vec[o:o + n], dtype=np.float64).reshape(shape)
        o += n
    assert o == vec.size
    return out


def flatten(params: dict) -> np.ndarray:
    return np.concatenate([np.asarray(params[n], np.float64).reshape(-1) for n, _ in SHAPES])


def bf16_round(x: np.ndarray) -> np.ndarray:
    """Round float32 values to bfloat16 (round to nearest even), returned as float64."""
    f = np.asarray(x, dtype=np.float32).copy()
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    u = ((u + 0x7FFF + lsb) >> 16) << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def encode(H: np.ndarray, res: float, cy: int, cx: int) -> np.ndarray:
    """The [3, 24, 24] input of the cell (cy, cx)."""
    Hh, Ww = H.shape

    def val(y, x):
        if 0 <= y < Hh and 0 <= x < Ww and np.isfinite(H[y, x]):
            return 1.0, float(H[y, x])
        return 0.0, 0.0

    X = np.zeros((3, PATCH, PATCH))
    for i in range(PATCH):
        for j in range(PATCH):
            y, x = cy - HALF + i, cx - HALF + j
            v, h = val(y, x)
            vx, hx = val(y, x + 1)
            vy, hy = val(y + 1, x)
            X[0, i, j] = v * vx * (hx - h) / res
            X[1, i, j] = v * vy * (hy - h) / res
            X[2, i, j] = v
    return X


def conv_stride2(X: np.ndarray, W: np.ndarray) -> np.ndarray:
    """Valid convolution (cross-correlation) with stride 2: X [B, C, n, n],
    W [O, C, k, k] -> [B, O, m, m] with m = (n - k) // 2 + 1."""
    B, C, n, _ = X.shape
    O, C2, k, _ = W.shape
    assert C == C2
    m = (n - k) // 2 + 1
    out = np.zeros((B, O, m, m))
    for i in range(k):
        for j in range(k):
            patch = X[:, :, i:i + 2 * m - 1:2, j:j + 2 * m - 1:2]      # [B, C, m, m]
            out += np.einsum("bcxy,oc->boxy", patch, W[:, :, i, j])
    return out


def conv_stride2_backward(X: np.ndarray, W: np.ndarray, dout: np.ndarray):
    B, C, n, _ = X.shape
    O, _, k, _ = W.shape
    m = dout.shape[-1]
    dX = np.zeros_like(X)
    dW = np.zeros_like(W)
    for i in range(k):
        for j in range(k):
            patch = X[:, :, i:i + 2 * m - 1:2, j:j + 2 * m - 1:2]
            dW[:, :, i, j] = np.einsum("bcxy,boxy->oc", patch, dout)
            dX[:, :, i:i + 2 * m - 1:2, j:j + 2 * m - 1:2] += np.einsum("boxy,oc->bcxy", dout,
                                                                        W[:, :, i, j])
    return dX, dW


def relu(x):
    return np.maximum(x, 0.0)


def _identity(x):
    return x


def forward(P: dict, X: np.ndarray, sc: np.ndarray, rnd=_identity):
    """X [B, 3, 24, 24], sc [B, 2] = (sin yaw, cos yaw) -> y [B, 4] and a cache.

    `rnd` is applied to every hidden activation (identity by default; pass
    bf16_round to mirror hardware that stores activations in bfloat16)."""
    B = X.shape[0]
    a1 = conv_stride2(X, P["W1"]) + P["b1"][None, :, None, None]
    o1 = rnd(relu(a1))
    a2 = conv_stride2(o1, P["W2"]) + P["b2"][None, :, None, None]
    o2 = rnd(relu(a2))
    f = o2.transpose(0, 2, 3, 1).reshape(B, 800)
    a3 = f @ P["W3"].T + sc @ P["Wy"].T + P["b3"]
    h1 = rnd(relu(a3))
    a4 = h1 @ P["W4"].T + P["b4"]
    h2 = rnd(relu(a4))
    y = h2 @ P["W5"].T + P["b5"]
    cache = dict(X=X, sc=sc, a1=a1, o1=o1, a2=a2, o2=o2, f=f, a3=a3, h1=h1, a4=a4, h2=h2)
    return y, cache


def backward(P: dict, cache: dict, dy: np.ndarray, rnd=_identity) -> dict:
    """Gradients of the loss in every parameter given dL/dy.  `rnd` is applied
    to the back-propagated deltas (identity by default)."""
    B = dy.shape[0]
    g = {}
    dy = rnd(dy)
    g["W5"] = dy.T @ cache["h2"]
    g["b5"] = dy.sum(0)
    da4 = rnd((dy @ P["W5"]) * (cache["a4"] > 0))
    g["W4"] = da4.T @ cache["h1"]
    g["b4"] = da4.sum(0)
    da3 = rnd((da4 @ P["W4"]) * (cache["a3"] > 0))
    g["W3"] = da3.T @ cache["f"]
    g["Wy"] = da3.T @ cache["sc"]
    g["b3"] = da3.sum(0)
    df = rnd((da3 @ P["W3"]) * (cache["f"] > 0))
    da2 = df.reshape(B, 5, 5, 32).transpose(0, 3, 1, 2)
    g["b2"] = da2.sum((0, 2, 3))
    do1, g["W2"] = conv_stride2_backward(cache["o1"], P["W2"], da2)
    da1 = rnd(do1 * (cache["a1"] > 0))
    g["b1"] = da1.sum((0, 2, 3))
    _, g["W1"] = conv_stride2_backward(cache["X"], P["W1"], da1)
    return g


LOSS_WEIGHTS = np.array([1.0, 1.0, 1.0, 1.0])


def loss(y: np.ndarray, t: np.ndarray, w: np.ndarray = LOSS_WEIGHTS):
    """Mean over the batch of sum_o w_o (y_o - t_o)^2, and its gradient in y."""
    B = y.shape[0]
    r = y - t
    L = float(np.sum(w[None, :] * r * r) / B)
    return L, 2.0 * w[None, :] * r / B


def _known(h) -> bool:
    return bool(np.isfinite(h)) and abs(float(h)) < 2.0 ** 60


def reference_height(H: np.ndarray, cy: int, cx: int):
    """Height the z output is expressed against: the cell's own height when
    known, else the mean of its known in-map 8-neighbours, else None (the state
    has no reference and is left to the plain method)."""
    if _known(H[cy, cx]):
        return float(H[cy, cx])
    vals = [float(H[y, x]) for y in range(cy - 1, cy + 2) for x in range(cx - 1, cx + 2)
            if (y, x) != (cy, cx) and 0 <= y < H.shape[0] and 0 <= x < H.shape[1]
            and _known(H[y, x])]
    return sum(vals) / len(vals) if vals else None


def targets(H: np.ndarray, z: float, roll: float, pitch: float, risk: float, cy: int, cx: int):
    """Scaled training targets of one state (which must have a reference height)."""
    return np.array([(z - reference_height(H, cy, cx)) / S_Z, roll / S_A, pitch / S_A, risk])


def adam_step(theta, grad, m, v, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (bias-corrected) of FP64 arrays; returns new (theta, m, v)."""
    m = b1 * m + (1 - b1) * grad
    v = b2 * v + (1 - b2) * grad * grad
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v
