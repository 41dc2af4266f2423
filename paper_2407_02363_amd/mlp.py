"""Thin ctypes binding of the surrogate entry points (include/sdf_mlp.h).

Argument marshalling only; every function forwards device pointers and the
current HIP stream to the C function of the same name.
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from .edt import EdtError, _check, _dev, _stream, lib as _edt_lib

JOINTS, N_IN, N_HIDDEN, N_OUT = 7, 14, 256, 12
IN_PAD, OUT_PAD = 32, 32
# offsets of the flat parameter block (must match sdf_mlp.h)
W1, B1, W2, B2, W3, B3, W4, B4, PARAMS = 0, 8192, 8448, 73984, 74240, 139776, 140032, 148224, 148256
LAYOUT = [(W1, B1, N_HIDDEN, IN_PAD), (W2, B2, N_HIDDEN, N_HIDDEN), (W3, B3, N_HIDDEN, N_HIDDEN),
          (W4, B4, OUT_PAD, N_HIDDEN)]
REAL = [(N_HIDDEN, N_IN), (N_HIDDEN, N_HIDDEN), (N_HIDDEN, N_HIDDEN), (N_OUT, N_HIDDEN)]

EXPORTED = ["sdf_mlp_workspace_bytes", "sdf_mlp_pack", "sdf_mlp_forward", "sdf_mlp_backward",
            "sdf_mlp_adam", "sdf_mlp_fallback", "sdf_mlp_calibrate", "sdf_mlp_select", "sdf_mlp_infer"]
_sig_done = False


def lib():
    global _sig_done
    L = _edt_lib()
    if not _sig_done:
        P, i32, f = ctypes.c_void_p, ctypes.c_int32, ctypes.c_float
        sig = {
            "sdf_mlp_workspace_bytes": ([i32], ctypes.c_size_t),
            "sdf_mlp_pack": ([P, P, P], ctypes.c_int),
            "sdf_mlp_forward": ([P, P, P, i32, P, i32, P, P, ctypes.c_size_t, P], ctypes.c_int),
            "sdf_mlp_backward": ([P, P, i32, P, i32, f, P, P, P, ctypes.c_size_t, P], ctypes.c_int),
            "sdf_mlp_adam": ([P, P, P, P, P, i32, f, f, f, f, P], ctypes.c_int),
            "sdf_mlp_fallback": ([P, P, P, i32, f, f, P, P, P], ctypes.c_int),
            "sdf_mlp_calibrate": ([P, P, i32, f, P, P], ctypes.c_int),
            "sdf_mlp_select": ([P, P, P, i32, i32, i32, P, P], ctypes.c_int),
            "sdf_mlp_infer": ([P, P, P, i32, P, P, P, f, f, P, P], ctypes.c_int),
        }
        for name, (args, res) in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _sig_done = True
    return L


def sdf_mlp_workspace_bytes(batch: int) -> int:
    return int(lib().sdf_mlp_workspace_bytes(int(batch)))


def new_workspace(batch: int, device="cuda"):
    return torch.empty(sdf_mlp_workspace_bytes(batch), dtype=torch.uint8, device=device)


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def sdf_mlp_pack(master, w16, stream=None):
    _check(lib().sdf_mlp_pack(_dev(master, torch.float32, "master", PARAMS),
                              _dev(w16, torch.bfloat16, "w16", PARAMS), _stream(stream)), "sdf_mlp_pack")


def _rows(t, width, name):
    if t.dim() != 2 or t.shape[1] != width:
        raise ValueError(f"{name}: expected shape [rows, {width}], got {tuple(t.shape)}")
    return t.shape[0]


def _idx(idx, batch):
    if idx is None:
        return None
    return _dev(idx, torch.int32, "idx", batch)


def sdf_mlp_forward(w16, master, q, y, ws, idx=None, stream=None):
    """q: float32 [R, 7]; idx: int32 [B] row indices into q (None: B = R);
    y: float32 [B, 12] or None."""
    rows = _rows(q, JOINTS, "q")
    b = rows if idx is None else idx.numel()
    _check(lib().sdf_mlp_forward(_dev(w16, torch.bfloat16, "w16", PARAMS),
                                 _dev(master, torch.float32, "master", PARAMS),
                                 _dev(q, torch.float32, "q", JOINTS * rows), rows, _idx(idx, b), b,
                                 None if y is None else _dev(y, torch.float32, "y", N_OUT * b),
                                 _ptr(ws), ws.numel(), _stream(stream)), "sdf_mlp_forward")


def sdf_mlp_infer(w16, master, q, y, radii=None, eps_vox=None, voxel=0.0, margin=0.0, need=None,
                  stream=None):
    """Predictions y float32 [B, 12] for q float32 [B, 7], one launch; with
    need (int32 [B]) also the fallback rule's decisions."""
    b = _rows(q, JOINTS, "q")
    _check(lib().sdf_mlp_infer(_dev(w16, torch.bfloat16, "w16", PARAMS),
                               _dev(master, torch.float32, "master", PARAMS),
                               _dev(q, torch.float32, "q", JOINTS * b), b,
                               _dev(y, torch.float32, "y", N_OUT * b),
                               _dev(radii, torch.float32, "radii", N_OUT),
                               _dev(eps_vox, torch.float32, "eps_vox", N_OUT), float(voxel), float(margin),
                               _dev(need, torch.int32, "need", b), _stream(stream)), "sdf_mlp_infer")


def sdf_mlp_backward(w16, target, grad, loss, ws, idx=None, clip_vox=0.0, stream=None):
    """target: float32 [R, 12]; idx: the same row indices as the forward."""
    rows = _rows(target, N_OUT, "target")
    b = rows if idx is None else idx.numel()
    _check(lib().sdf_mlp_backward(_dev(w16, torch.bfloat16, "w16", PARAMS),
                                  _dev(target, torch.float32, "target", N_OUT * rows), rows,
                                  _idx(idx, b), b, float(clip_vox),
                                  _dev(grad, torch.float32, "grad", PARAMS),
                                  None if loss is None else _dev(loss, torch.float32, "loss", 1),
                                  _ptr(ws), ws.numel(), _stream(stream)), "sdf_mlp_backward")


def sdf_mlp_adam(master, w16, m, v, grad, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8,
                 stream=None):
    _check(lib().sdf_mlp_adam(_dev(master, torch.float32, "master", PARAMS),
                              _dev(w16, torch.bfloat16, "w16", PARAMS),
                              _dev(m, torch.float32, "m", PARAMS), _dev(v, torch.float32, "v", PARAMS),
                              _dev(grad, torch.float32, "grad", PARAMS), int(step), float(lr),
                              float(beta1), float(beta2), float(eps), _stream(stream)), "sdf_mlp_adam")


def sdf_mlp_fallback(y, radii, eps_vox, voxel, margin, need, count, stream=None):
    """eps_vox: float32 [12] device tensor (per-sphere error bound, voxels)."""
    b = y.shape[0]
    _check(lib().sdf_mlp_fallback(_dev(y, torch.float32, "y", N_OUT * b),
                                  _dev(radii, torch.float32, "radii", N_OUT),
                                  _dev(eps_vox, torch.float32, "eps_vox", N_OUT), b, float(voxel),
                                  float(margin), _dev(need, torch.int32, "need", b),
                                  _dev(count, torch.int32, "count", 1), _stream(stream)),
           "sdf_mlp_fallback")


def sdf_mlp_select(y, need, exact, out, stream=None):
    """out[b] = exact[b] where need[b] != 0, else y[b]; exact is a float32
    device view [batch, 12] with any strides (e.g. the dist_vox words of
    sphere query records), y and out contiguous [batch, 12]."""
    b = y.shape[0]
    if exact.dtype != torch.float32 or not exact.is_cuda or tuple(exact.shape) != (b, N_OUT):
        raise ValueError("exact must be a float32 device view of shape [batch, 12]")
    _check(lib().sdf_mlp_select(_dev(y, torch.float32, "y", N_OUT * b),
                                _dev(need, torch.int32, "need", b),
                                ctypes.c_void_p(exact.data_ptr()), exact.stride(0), exact.stride(1), b,
                                _dev(out, torch.float32, "out", N_OUT * b), _stream(stream)),
           "sdf_mlp_select")


def sdf_mlp_calibrate(pred, target, clip_vox, eps_vox, stream=None):
    """eps_vox (float32 [12], device) = per-sphere largest overestimate on
    the rows whose target lies below clip_vox."""
    b = pred.shape[0]
    _check(lib().sdf_mlp_calibrate(_dev(pred, torch.float32, "pred", N_OUT * b),
                                   _dev(target, torch.float32, "target", N_OUT * b), b,
                                   float(clip_vox), _dev(eps_vox, torch.float32, "eps_vox", N_OUT),
                                   _stream(stream)), "sdf_mlp_calibrate")


def unpack(master_np: np.ndarray):
    """[(W, b)] with the padding stripped, from a flat parameter block."""
    out = []
    for (wo, bo, rows, cols), (ro, ci) in zip(LAYOUT, REAL):
        W = master_np[wo:wo + rows * cols].reshape(rows, cols)[:ro, :ci]
        out.append((W.astype(np.float64), master_np[bo:bo + ro].astype(np.float64)))
    return out


def init_params(seed: int) -> np.ndarray:
    """Flat float32 block: He-uniform weights (bound sqrt(6 / fan_in)), zero
    biases, zero padding."""
    g = np.random.Generator(np.random.PCG64(seed))
    p = np.zeros(PARAMS, np.float32)
    for (wo, bo, rows, cols), (ro, ci) in zip(LAYOUT, REAL):
        bound = np.sqrt(6.0 / ci)
        W = np.zeros((rows, cols), np.float32)
        W[:ro, :ci] = g.uniform(-bound, bound, size=(ro, ci))
        p[wo:wo + rows * cols] = W.ravel()
    return p


__all__ = EXPORTED + ["EdtError", "init_params", "unpack", "new_workspace", "LAYOUT", "PARAMS"]
