"""Training driver for the learned surrogate.

Labels come from the plain HIP kernel (seb_assess_se2) on seeded training
terrains; every training step runs in the library's kernels (seb_net_train_step).
This module only assembles the data on the device and loops.
"""
from __future__ import annotations

import numpy as np

from . import inputs as I
from . import seb


def has_reference(maps: np.ndarray) -> np.ndarray:
    """Cells of [n][H][W] height maps whose state has a height reference for
    the network's z output: the cell or one of its in-map 8-neighbours known."""
    known = np.isfinite(maps) & (np.abs(maps) < 2.0 ** 60)
    pad = np.pad(known, ((0, 0), (1, 1), (1, 1)))
    H, W = maps.shape[1:]
    out = np.zeros_like(known)
    for dy in range(3):
        for dx in range(3):
            out |= pad[:, dy:dy + H, dx:dx + W]
    return out


class TrainingData:
    """Training maps, their plain-method labels and the sample list, on the GPU."""

    def __init__(self, seeds=I.SURROGATE_TRAIN_SEEDS, params=I.SURROGATE_LABEL_PARAMS,
                 sample_seed: int = 4, count: int | None = None):
        import torch
        self.params = params
        maps = np.stack([I.surrogate_training_map(s, params.width, params.resolution)
                         for s in seeds])
        self.maps = torch.from_numpy(maps).cuda()
        n, K = len(seeds), params.n_yaw
        self.labels = {k: torch.empty((n, K, params.height, params.width), dtype=torch.float32,
                                      device="cuda") for k in ("z", "roll", "pitch", "risk")}
        status = torch.empty((n, K, params.height, params.width), dtype=torch.uint8, device="cuda")
        with seb.Context(params) as ctx:
            for i in range(n):
                out = {k: self.labels[k][i] for k in self.labels}
                out["status"] = status[i]
                ctx.assess(self.maps[i], out)
        torch.cuda.synchronize()
        # Samples: yaw bins of the first half (the second half mirrors them),
        # every cell (windows may reach past the map edge) with a reference
        # height (own cell or an 8-neighbour known), plain fit valid.
        cand = I.surrogate_samples(n, params.width, K // 2 if K % 2 == 0 else K, sample_seed)
        st = status.cpu().numpy()
        ok = (st[cand[:, 0], cand[:, 3], cand[:, 1], cand[:, 2]] & seb.ST_VALID) > 0
        ok &= has_reference(maps)[cand[:, 0], cand[:, 1], cand[:, 2]]
        cand = cand[ok]
        if count is not None:
            cand = cand[:count]
        self.samples = torch.from_numpy(np.ascontiguousarray(cand)).cuda()
        self.n_samples = len(cand)

    def batch(self, step: int, size: int):
        n = self.n_samples - self.n_samples % size
        i0 = (step * size) % n
        return self.samples[i0:i0 + size]


def pool2(maps: np.ndarray, py: int, px: int) -> np.ndarray:
    """2 x 2 average pooling of [n][H][W] height maps, blocks starting at cell
    (py, px) (0 or 1): pooled cell (Y, X), Y < ceil(H / 2), X < ceil(W / 2),
    covers cells (2Y + py + {0, 1}, 2X + px + {0, 1}) and holds the mean of
    their known in-map heights, NaN if none is known."""
    n, H, W = maps.shape
    Hp, Wp = (H + 1) // 2, (W + 1) // 2
    m = np.full((n, 2 * Hp + 2, 2 * Wp + 2), np.nan)
    m[:, :H, :W] = maps
    m = m[:, py:py + 2 * Hp, px:px + 2 * Wp]
    known = np.isfinite(m) & (np.abs(m) < 2.0 ** 60)
    v = np.where(known, m, 0.0).reshape(n, Hp, 2, Wp, 2).sum(axis=(2, 4))
    c = known.reshape(n, Hp, 2, Wp, 2).sum(axis=(2, 4))
    with np.errstate(invalid="ignore", divide="ignore"):
        return np.where(c > 0, v / np.maximum(c, 1), np.nan).astype(np.float32)


class PooledTrainingData:
    """Training data for a footprint larger than the network's 24 x 24 window
    at the map's resolution: each state's 48 x 48-cell window is 2 x 2
    average-pooled to 24 x 24 cells of twice the size.  The states of cells
    of parity (py, px) are the cells of the pooled map of that parity, so each
    full-resolution map gives four pooled maps (at twice the resolution) and
    labels re-indexed to them; the network then sees ordinary 24 x 24 windows
    and its z output is relative to the pooled cell's reference height.
    Labels are the plain kernel's, on the full-resolution maps."""

    def __init__(self, maps: np.ndarray, params, sample_seed: int = 5, count: int | None = None):
        import torch
        n, H, W = maps.shape
        assert (H, W) == (params.height, params.width) and H % 2 == 0 and W % 2 == 0
        K = params.n_yaw
        full = {k: np.empty((n, K, H, W), np.float32) for k in ("z", "roll", "pitch", "risk")}
        status = np.empty((n, K, H, W), np.uint8)
        with seb.Context(params) as ctx:
            for i in range(n):
                out = ctx.assess(torch.from_numpy(maps[i]).cuda())
                for k in full:
                    full[k][i] = out[k].cpu().numpy()
                status[i] = out["status"].cpu().numpy()
        pooled, labels, st = [], {k: [] for k in full}, []
        for py in range(2):
            for px in range(2):
                pooled.append(pool2(maps, py, px))
                for k in full:
                    labels[k].append(full[k][:, :, py::2, px::2])
                st.append(status[:, :, py::2, px::2])
        # pooled map index = (parity * n + map)
        pm = np.concatenate(pooled)
        self.params = params.with_(width=W // 2, height=H // 2, resolution=2 * params.resolution)
        self.maps = torch.from_numpy(np.ascontiguousarray(pm)).cuda()
        self.labels = {k: torch.from_numpy(np.ascontiguousarray(np.concatenate(v))).cuda()
                       for k, v in labels.items()}
        stp = np.concatenate(st)
        U = K // 2 if K % 2 == 0 else K
        cand = I.surrogate_samples(len(pm), W // 2, U, sample_seed)
        ok = (stp[cand[:, 0], cand[:, 3], cand[:, 1], cand[:, 2]] & seb.ST_VALID) > 0
        ok &= has_reference(pm)[cand[:, 0], cand[:, 1], cand[:, 2]]
        cand = cand[ok]
        if count is not None:
            cand = cand[:count]
        self.samples = torch.from_numpy(np.ascontiguousarray(cand)).cuda()
        self.n_samples = len(cand)

    batch = TrainingData.batch


def validation_loss(net: "seb.Net", data: TrainingData, batch: int = 4096) -> float:
    """Mean training loss over every sample of `data` (whole batches), with
    the weights left unchanged (the library's training step in its
    gradient-only mode)."""
    import torch
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    grad = torch.empty(seb.Net.param_count(), dtype=torch.float32, device="cuda")
    p = data.params
    total, n = 0.0, data.n_samples // batch
    for i in range(n):
        net.train_step(data.maps, data.labels, data.samples[i * batch:(i + 1) * batch],
                       p.resolution, p.n_yaw, 0.0, loss=loss, grad=grad)
        total += float(loss.item())
    return total / max(1, n)


def train(net: "seb.Net", data: TrainingData, steps: int, batch: int = 4096,
          lr: float = 2e-3, lr_final: float = 1e-4, log_every: int = 0):
    """Adam with a cosine learning-rate decay; returns the loss history (host floats)."""
    import math
    import torch
    p = data.params
    loss = torch.zeros(steps, dtype=torch.float32, device="cuda")
    for s in range(steps):
        frac = s / max(1, steps - 1)
        lr_s = lr_final + 0.5 * (lr - lr_final) * (1 + math.cos(math.pi * frac))
        net.train_step(data.maps, data.labels, data.batch(s, batch), p.resolution, p.n_yaw,
                       lr_s, loss=loss[s:s + 1])
        if log_every and (s + 1) % log_every == 0:
            print(f"step {s + 1}: loss {float(loss[s]):.5f}", flush=True)
    return loss.cpu().numpy()
