"""ctypes binding of the task-priority controller (include/controller.h).

Argument marshalling only: numpy float64 arrays in, the library's tp_step
does the work on the host."""
from __future__ import annotations

import ctypes

import numpy as np

from .edt import EdtError, lib as _edt_lib


class TpParams(ctypes.Structure):
    _fields_ = [("buffer", ctypes.c_double), ("target_offset", ctypes.c_double),
                ("gain", ctypes.c_double), ("reg_max", ctypes.c_double),
                ("reg_width", ctypes.c_double), ("pinv_tol", ctypes.c_double)]


EXPORTED = ["tp_step"]
_sig = False


def lib():
    global _sig
    L = _edt_lib()
    if not _sig:
        P = ctypes.c_void_p
        L.tp_step.argtypes = [ctypes.c_int32, P, P, ctypes.c_int32, P, P, P, P, P,
                              ctypes.POINTER(TpParams), P, P, P]
        L.tp_step.restype = ctypes.c_int
        _sig = True
    return L


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def tp_step(axes, origins, count, C, O, x_m, qdot0=None, buffer=0.02, target_offset=0.05, gain=2.0,
            reg_max=1e-3, reg_width=1e-2, pinv_tol=1e-12):
    """One control step: (qdot [n], activation [m], x [m])."""
    axes = np.ascontiguousarray(axes, np.float64)
    origins = np.ascontiguousarray(origins, np.float64)
    n = axes.shape[0]
    C = np.ascontiguousarray(C, np.float64).reshape(-1, 3)
    O = np.ascontiguousarray(O, np.float64).reshape(-1, 3)
    m = C.shape[0]
    cnt = np.ascontiguousarray(count, np.int32)
    xm = np.ascontiguousarray(np.broadcast_to(np.asarray(x_m, np.float64), (m,)))
    q0 = None if qdot0 is None else np.ascontiguousarray(qdot0, np.float64)
    qdot = np.zeros(n)
    act = np.zeros(m)
    x = np.zeros(m)
    prm = TpParams(buffer, target_offset, gain, reg_max, reg_width, pinv_tol)
    rc = lib().tp_step(n, _p(axes), _p(origins), m, _p(cnt), _p(C), _p(O), _p(xm), _p(q0),
                       ctypes.byref(prm), _p(qdot), _p(act), _p(x))
    if rc != 0:
        raise EdtError(rc, "tp_step", lib().edt_last_error().decode())
    return qdot, act, x
