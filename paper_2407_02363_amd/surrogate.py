"""Learned self-distance surrogate: training and fallback driver.

Holds the flat FP32 master parameters, their BF16 copy, the Adam moments,
the gradient block and the workspaces on the device, and drives the
library's kernels (sdf_mlp_forward / _backward / _adam / _fallback).  The
labels come from the exact self-map EDT (selfmap.SelfMapLabeler); the
surrogate's worst error on held-out states, in voxels, sets how wide the
band around the safety margin is inside which the exact EDT stays in
charge.
"""
from __future__ import annotations

import numpy as np
import torch

from . import mlp


class Surrogate:
    def __init__(self, device="cuda:0", seed: int = 0, batch: int = 4096):
        self.dev = torch.device(device)
        d = self.dev
        self.batch = int(batch)
        self.master = torch.from_numpy(mlp.init_params(seed)).to(d)
        self.w16 = torch.empty(mlp.PARAMS, dtype=torch.bfloat16, device=d)
        self.m = torch.zeros(mlp.PARAMS, dtype=torch.float32, device=d)
        self.v = torch.zeros(mlp.PARAMS, dtype=torch.float32, device=d)
        self.grad = torch.zeros(mlp.PARAMS, dtype=torch.float32, device=d)
        self.loss = torch.zeros(1, dtype=torch.float32, device=d)
        self.ws = mlp.new_workspace(self.batch, d)
        self.step = 0
        mlp.sdf_mlp_pack(self.master, self.w16)

    def train_step(self, q, target, lr=1e-3):
        """One forward / backward / Adam step on a minibatch (device tensors)."""
        mlp.sdf_mlp_forward(self.w16, self.master, q, None, self.ws)
        mlp.sdf_mlp_backward(self.w16, target, self.grad, self.loss, self.ws)
        self.step += 1
        mlp.sdf_mlp_adam(self.master, self.w16, self.m, self.v, self.grad, self.step, lr)

    def train(self, q, target, epochs: int, lr: float = 1e-3, seed: int = 0, log=None):
        """Minibatch training; q float32 [N, 7], target float32 [N, 12] on
        the device.  Returns the mean loss of every epoch."""
        n = q.shape[0]
        g = torch.Generator(device="cpu").manual_seed(seed)
        hist = []
        for ep in range(epochs):
            perm = torch.randperm(n, generator=g).to(self.dev)
            total = torch.zeros(1, dtype=torch.float32, device=self.dev)
            steps = 0
            for s0 in range(0, n - self.batch + 1, self.batch):
                idx = perm[s0:s0 + self.batch]
                self.train_step(q[idx].contiguous(), target[idx].contiguous(), lr)
                total += self.loss
                steps += 1
            hist.append(float(total.item()) / max(1, steps))
            if log:
                log(f"epoch {ep}: loss {hist[-1]:.4f}")
        return hist

    def predict(self, q, out=None):
        """Predicted distances (voxels) float32 [N, 12] for q float32 [N, 7]."""
        n = q.shape[0]
        y = out if out is not None else torch.empty((n, mlp.N_OUT), dtype=torch.float32, device=self.dev)
        for s0 in range(0, n, self.batch):
            k = min(self.batch, n - s0)
            mlp.sdf_mlp_forward(self.w16, self.master, q[s0:s0 + k], y[s0:s0 + k], self.ws)
        return y

    def fallback(self, y, radii, voxel, margin, eps_vox, need=None, count=None):
        n = y.shape[0]
        need = need if need is not None else torch.empty(n, dtype=torch.int32, device=self.dev)
        count = count if count is not None else torch.empty(1, dtype=torch.int32, device=self.dev)
        mlp.sdf_mlp_fallback(y, radii, voxel, margin, eps_vox, need, count)
        return need, count

    def state(self) -> dict:
        return {"master": self.master.cpu().numpy(), "m": self.m.cpu().numpy(),
                "v": self.v.cpu().numpy(), "step": self.step}

    def load(self, st: dict):
        self.master.copy_(torch.from_numpy(np.asarray(st["master"], np.float32)))
        self.m.copy_(torch.from_numpy(np.asarray(st["m"], np.float32)))
        self.v.copy_(torch.from_numpy(np.asarray(st["v"], np.float32)))
        self.step = int(st["step"])
        mlp.sdf_mlp_pack(self.master, self.w16)
