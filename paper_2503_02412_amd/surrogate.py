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
