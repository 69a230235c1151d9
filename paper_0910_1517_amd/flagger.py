"""Training driver of the learned RFI flagger.

The host only draws the random numbers (initial weights, mini-batch tile
lists) and sequences the calls; every forward, backward and Adam step runs in
the library's kernels (corr_cnn_train_step), inference in the fused kernel
(corr_cnn_infer).
"""
from __future__ import annotations

import numpy as np

from . import CNN, CNN_PARAMS, cnn_infer, cnn_tiles

# (Cout, Cin) of the three 3x3 layers, in parameter order
LAYERS = ((16, 1), (16, 16), (1, 16))


def init_params(seed: int) -> np.ndarray:
    """He-normal weights (std sqrt(2 / (9 Cin))) and zero biases, float32."""
    g = np.random.Generator(np.random.Philox(np.random.SeedSequence([int(seed) & 0xFFFFFFFF, 0xC11])))
    parts = []
    for co, ci in LAYERS:
        parts.append(g.standard_normal(co * ci * 9) * np.sqrt(2.0 / (9 * ci)))
        parts.append(np.zeros(co))
    p = np.concatenate(parts).astype(np.float32)
    assert p.size == CNN_PARAMS
    return p


class Flagger:
    """Parameters, Adam state and the training handle on one device."""

    def __init__(self, *, seed: int = 0, batch: int = 16, lr: float = 2e-3, device="cuda"):
        import torch
        self.device = device
        self.params = torch.from_numpy(init_params(seed)).to(device)
        self.m = torch.zeros(CNN_PARAMS, device=device)
        self.v = torch.zeros(CNN_PARAMS, device=device)
        self.step = 0
        self.batch = batch
        self.cnn = CNN(batch, lr=lr, device=device)
        self.rng = np.random.Generator(np.random.Philox(np.random.SeedSequence([int(seed) & 0xFFFFFFFF, 0xB47])))

    def train(self, power, labels, steps: int):
        """`steps` Adam steps on mini-batches of `batch` tiles drawn uniformly
        without replacement from power [S][T][C] (device float32) with MAD
        labels [S][T][C] (device uint8).  Returns the per-step losses (numpy)."""
        import torch
        S, T, C = power.shape
        n = cnn_tiles(S, T, C)
        b = min(self.batch, n)
        lists = np.stack([self.rng.choice(n, b, replace=False) for _ in range(steps)]).astype(np.int32)
        tiles = torch.from_numpy(lists).to(self.device)
        losses = torch.zeros(steps, device=self.device)
        for k in range(steps):
            self.step += 1
            self.cnn.train_step(self.params, self.m, self.v, self.step, power, labels, tiles[k], losses[k:k + 1])
        self.cnn.check_device_errors()
        return losses.cpu().numpy()

    def infer(self, power, flags, *, threshold: float = 0.5, logits=None, guard: float = 0.0):
        """Flags of power [S][T][C]; guard > 0 adds the MAD column guard at M = guard."""
        cnn_infer(self.params, power, flags, threshold=threshold, logits=logits, guard=guard)
