"""CPU oracle of the learned self-distance surrogate -- TEST INFRASTRUCTURE ONLY.

The surrogate maps a joint state to the distance (in voxels) between each of
12 arm bounding spheres and the self-collision obstacle set, i.e. the task
variable x_s of Eq. selftaskvar that the exact self-map EDT measures
(Sec. III-E).  The network: input [sin q1, cos q1, ..., sin q7, cos q7]
(14 values) -> 256 -> 256 -> 256 -> 12, ReLU between layers, trained with
mean squared error and Adam.  The paper has no such network; this oracle
defines what the device kernels compute, in numpy with float64 arithmetic:

  rounding=True   the device's precision plan: inputs, weights and hidden
                  activations rounded to bfloat16 (round to nearest even),
                  products summed exactly (float64), float32 biases, the
                  result of every sum rounded to float32 before any bf16
                  rounding; backward rounds dY and every masked gradient to
                  bf16 before it feeds a product, as the device does.
  rounding=False  the same network in plain float64 (pinned against torch
                  autograd and finite differences in the tests).

Weights are kept as W[out][in] (PyTorch convention).
"""
from __future__ import annotations

import numpy as np

N_IN, N_HID, N_OUT = 14, 256, 12
LAYERS = [(N_IN, N_HID), (N_HID, N_HID), (N_HID, N_HID), (N_HID, N_OUT)]


def f32(x):
    return np.asarray(x, np.float64).astype(np.float32).astype(np.float64)


def bf16(x):
    """Round float64 values to bfloat16 (nearest even), via float32."""
    a = np.asarray(x, np.float64).astype(np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    nan = np.isnan(a)
    lsb = (u >> 16) & 1
    u = (u + 0x7FFF + lsb) & 0xFFFF0000
    out = u.astype(np.uint32).view(np.float32).astype(np.float64)
    return np.where(nan, np.nan, out)


def encode(q, rounding=True):
    """[sin q1, cos q1, ..., sin q7, cos q7] for q of shape [B, 7]."""
    q = np.asarray(q, np.float64)
    x = np.empty((q.shape[0], 2 * q.shape[1]))
    x[:, 0::2] = np.sin(q)
    x[:, 1::2] = np.cos(q)
    return bf16(x) if rounding else x


def forward(params, q, rounding=True):
    """params: list of (W, b).  Returns (y, acts) with acts = [x, h1, h2, h3]."""
    x = encode(q, rounding)
    acts = [x]
    h = x
    for li, (W, b) in enumerate(params):
        z = h @ W.T + b
        if rounding:
            z = f32(z)
        if li < len(params) - 1:
            h = np.maximum(z, 0.0)
            if rounding:
                h = bf16(h)
            acts.append(h)
        else:
            y = z
    return y, acts


def loss_and_dy(y, target, rounding=True, clip=None):
    """MSE over every output; dY = 2 (y - t) / (B * 12).  With clip > 0 the
    targets are min(target, clip) first (the network learns the distance
    saturated at clip)."""
    if clip is not None and clip > 0:
        target = np.minimum(target, clip)
    d = y - target
    loss = float(np.mean(d * d))
    dy = 2.0 * d / d.size
    return loss, (bf16(f32(dy)) if rounding else dy)


def backward(params, acts, dy, rounding=True):
    """Gradients [(dW, db)] per layer for upstream gradient dy of the output.

    dW_l = dP_l^T h_{l-1}, db_l = sum over the batch of dP_l, and the
    upstream gradient of layer l-1 is (dP_l W_l) masked where h_{l-1} > 0.
    """
    grads = [None] * len(params)
    dp = dy
    for li in range(len(params) - 1, -1, -1):
        W, _ = params[li]
        h_prev = acts[li]
        dW = dp.T @ h_prev
        db = dp.sum(axis=0)
        if rounding:
            dW, db = f32(dW), f32(db)
        grads[li] = (dW, db)
        if li > 0:
            g = dp @ W
            if rounding:
                g = f32(g)
            g = np.where(h_prev > 0, g, 0.0)
            dp = bf16(g) if rounding else g
    return grads


def adam(master, grads, m, v, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (bias-corrected) on lists of float arrays; returns new
    (master, m, v).  step counts from 1."""
    out_w, out_m, out_v = [], [], []
    c1 = 1.0 - b1 ** step
    c2 = 1.0 - b2 ** step
    for w, g, mm, vv in zip(master, grads, m, v):
        mm = b1 * mm + (1.0 - b1) * g
        vv = b2 * vv + (1.0 - b2) * g * g
        w = w - lr * (mm / c1) / (np.sqrt(vv / c2) + eps)
        out_w.append(w)
        out_m.append(mm)
        out_v.append(vv)
    return out_w, out_m, out_v


def needs_exact(pred_vox, radii_m, voxel, margin_m, eps_vox):
    """Exact-EDT fallback rule: a state needs the exact self-map transform when
    any sphere's predicted clearance, pred * voxel - r, is below the safety
    margin plus the surrogate's error bound for that sphere (eps_vox: one
    number or one per sphere, voxels), or is not a number.

    The rule turns floats into a yes/no, so it is evaluated in float32 with
    one rounding per operation in this order -- c = pred * voxel - r and
    t = margin + eps * voxel -- the precision and order of the device's
    decision."""
    one = np.float32
    pred = np.asarray(pred_vox, np.float32)
    r = np.asarray(radii_m, np.float32)[None, :]
    eps = np.broadcast_to(np.asarray(eps_vox, np.float32), (pred.shape[1],))[None, :]
    with np.errstate(invalid="ignore"):
        c = pred * one(voxel) - r
        t = one(margin_m) + eps * one(voxel)
        # a NaN prediction is never trusted
        return (~(c >= t)).any(axis=1)


def calibrate(pred_vox, target_vox, clip_vox):
    """Per-sphere error bound the fallback rule allows for: the largest
    overestimate pred - target (float32 difference) over the held-out rows
    whose exact target lies below clip_vox (every row if clip_vox <= 0),
    and 0 if there is none.  Only an overestimate can hide a sphere inside
    the margin, and such a sphere has an exact distance below the clip when
    (margin + radius) / voxel + bound < clip_vox.  A NaN prediction on a
    counted row makes the bound infinite."""
    pred = np.asarray(pred_vox, np.float32)
    tgt = np.asarray(target_vox, np.float32)
    with np.errstate(invalid="ignore"):
        rows = np.ones(tgt.shape, bool) if clip_vox <= 0 else (tgt < np.float32(clip_vox))
        d = pred - tgt
    d = np.where(np.isnan(pred), np.float32(np.inf), d)
    d = np.where(rows, d, np.float32(0.0))
    return np.maximum(d.max(axis=0), np.float32(0.0)).astype(np.float32)
