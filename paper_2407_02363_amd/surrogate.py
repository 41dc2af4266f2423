"""Learned self-distance surrogate: training and fallback driver.

Holds the flat FP32 master parameters, their BF16 copy, the Adam moments,
the gradient block and the workspaces on the device, and drives the
library's kernels (sdf_mlp_forward / _backward / _adam / _fallback).  The
labels come from the exact self-map EDT (selfmap.SelfMapLabeler).  The
network learns the distance saturated at clip_vox (only distances near the
safety margin decide anything), and its largest overestimate per sphere on
held-out states (calibrate), in voxels, sets how wide the band above the
safety margin is inside which the exact EDT stays in charge.
"""
from __future__ import annotations

import math

import numpy as np
import torch

from . import mlp


class Surrogate:
    def __init__(self, device="cuda:0", seed: int = 0, batch: int = 4096, clip_vox: float = 24.0):
        self.dev = torch.device(device)
        d = self.dev
        self.batch = int(batch)
        self.clip_vox = float(clip_vox)
        self.eps = torch.full((mlp.N_OUT,), float("inf"), dtype=torch.float32, device=d)
        self.master = torch.from_numpy(mlp.init_params(seed)).to(d)
        self.w16 = torch.empty(mlp.PARAMS, dtype=torch.bfloat16, device=d)
        self.m = torch.zeros(mlp.PARAMS, dtype=torch.float32, device=d)
        self.v = torch.zeros(mlp.PARAMS, dtype=torch.float32, device=d)
        self.grad = torch.zeros(mlp.PARAMS, dtype=torch.float32, device=d)
        self.loss = torch.zeros(1, dtype=torch.float32, device=d)
        self.ws = mlp.new_workspace(self.batch, d)
        self.step = 0
        mlp.sdf_mlp_pack(self.master, self.w16)

    def train_step(self, q, target, lr=1e-3, idx=None):
        """One forward / backward / Adam step on the minibatch idx (int32
        device tensor of rows of q and target; None = all rows)."""
        mlp.sdf_mlp_forward(self.w16, self.master, q, None, self.ws, idx=idx)
        mlp.sdf_mlp_backward(self.w16, target, self.grad, self.loss, self.ws, idx=idx,
                             clip_vox=self.clip_vox)
        self.step += 1
        mlp.sdf_mlp_adam(self.master, self.w16, self.m, self.v, self.grad, self.step, lr)

    def train(self, q, target, epochs: int, lr: float = 1e-3, seed: int = 0, log=None,
              lr_final: float | None = None):
        """Minibatch training; q float32 [N, 7], target float32 [N, 12] on
        the device.  Returns the mean loss of every epoch.  With lr_final
        the step size follows a cosine from lr down to lr_final over all
        steps, else it stays at lr."""
        n = q.shape[0]
        g = torch.Generator(device="cpu").manual_seed(seed)
        hist = []
        per_epoch = max(0, (n - self.batch) // self.batch + 1)
        total_steps = max(1, epochs * per_epoch)
        k = 0
        for ep in range(epochs):
            perm = torch.randperm(n, generator=g).to(torch.int32).to(self.dev)
            total = torch.zeros(1, dtype=torch.float32, device=self.dev)
            steps = 0
            for s0 in range(0, n - self.batch + 1, self.batch):
                idx = perm[s0:s0 + self.batch]
                a = lr
                if lr_final is not None:
                    a = lr_final + 0.5 * (lr - lr_final) * (1.0 + math.cos(math.pi * k / total_steps))
                k += 1
                self.train_step(q, target, a, idx=idx)
                total += self.loss
                steps += 1
            hist.append(float(total.item()) / max(1, steps))
            if log:
                log(f"epoch {ep}: loss {hist[-1]:.4f}")
        return hist

    def predict(self, q, out=None):
        """Predicted distances (voxels) float32 [N, 12] for q float32 [N, 7]
        (the one-launch inference kernel; the same bits as the forward pass)."""
        n = q.shape[0]
        y = out if out is not None else torch.empty((n, mlp.N_OUT), dtype=torch.float32, device=self.dev)
        if n:
            mlp.sdf_mlp_infer(self.w16, self.master, q, y)
        return y

    def calibrate(self, q, target):
        """Per-sphere error bound (voxels) from held-out states with exact
        labels: kept in self.eps for fallback() and returned."""
        p = self.predict(q)
        mlp.sdf_mlp_calibrate(p, target, self.clip_vox, self.eps)
        return self.eps

    def fallback(self, y, radii, voxel, margin, eps_vox=None, need=None, count=None):
        """eps_vox: float32 [12] device tensor (None = self.eps), or a
        number used for every sphere."""
        n = y.shape[0]
        if eps_vox is None:
            eps_vox = self.eps
        elif not isinstance(eps_vox, torch.Tensor):
            eps_vox = torch.full((mlp.N_OUT,), float(eps_vox), dtype=torch.float32, device=self.dev)
        need = need if need is not None else torch.empty(n, dtype=torch.int32, device=self.dev)
        count = count if count is not None else torch.empty(1, dtype=torch.int32, device=self.dev)
        mlp.sdf_mlp_fallback(y, radii, eps_vox, voxel, margin, need, count)
        return need, count

    def state(self) -> dict:
        return {"master": self.master.cpu().numpy(), "m": self.m.cpu().numpy(),
                "v": self.v.cpu().numpy(), "step": self.step, "eps": self.eps.cpu().numpy(),
                "clip_vox": self.clip_vox}

    def load(self, st: dict):
        self.master.copy_(torch.from_numpy(np.asarray(st["master"], np.float32)))
        self.m.copy_(torch.from_numpy(np.asarray(st["m"], np.float32)))
        self.v.copy_(torch.from_numpy(np.asarray(st["v"], np.float32)))
        self.step = int(st["step"])
        if "eps" in st:
            self.eps.copy_(torch.from_numpy(np.asarray(st["eps"], np.float32)))
        self.clip_vox = float(st.get("clip_vox", self.clip_vox))
        mlp.sdf_mlp_pack(self.master, self.w16)


class AssistedLookahead:
    """One look-ahead batch of S joint states with no host round trip: the
    surrogate predicts every state's sphere distances and, in the same launch
    (sdf_mlp_infer), marks by the fallback rule the states it cannot clear;
    the labeler's gated transform runs the exact
    self-map EDT for those states only (the others' work-groups return at
    once), and sdf_mlp_select keeps the exact distances of the marked states
    and the predictions of the rest.  The whole batch is one HIP graph.

    labeler: a SelfMapLabeler whose full chunk is S states; its gate buffer
    receives the fallback flags.  The distances are those of the states last
    staged with run(); the result buffer is overwritten by every run."""

    def __init__(self, sur: Surrogate, labeler, radii, voxel: float, margin: float,
                 use_graph: bool = True):
        self.sur = sur
        self.lab = labeler
        S = labeler.chunk
        self.S = S
        d = sur.dev
        self.radii = radii
        self.voxel = float(voxel)
        self.margin = float(margin)
        self.q = torch.zeros((S, mlp.JOINTS), dtype=torch.float32, device=d)
        self.y = torch.empty((S, mlp.N_OUT), dtype=torch.float32, device=d)
        self.out = torch.empty((S, mlp.N_OUT), dtype=torch.float32, device=d)
        self.need = labeler.gate[:S]
        self.graph = None
        if use_graph:
            self._body()
            torch.cuda.synchronize(d)
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g, capture_error_mode="thread_local"):
                self._body()
            torch.cuda.synchronize(d)
            self.graph = g

    def _body(self):
        s = self.sur
        mlp.sdf_mlp_infer(s.w16, s.master, self.q, self.y, self.radii, s.eps, self.voxel, self.margin,
                          self.need)
        self.lab.run_chunk(self.S, gated=True)
        mlp.sdf_mlp_select(self.y, self.need, self.lab.exact_view(self.S), self.out)

    def run(self, q, poses, centres):
        """q float32 [S, 7], poses / centres as SelfMapLabeler.stage gives
        them (device).  Returns the [S, 12] distances (voxels, device); need
        (int32 [S]) holds which states took the exact path."""
        self.q.copy_(q)
        self.lab.poses[:self.S].copy_(poses)
        self.lab.centres[:self.S].copy_(centres)
        if self.graph is not None:
            self.graph.replay()
        else:
            self._body()
        return self.out
