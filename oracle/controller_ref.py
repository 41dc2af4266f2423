"""CPU oracle of the task-priority collision-avoidance controller --
TEST INFRASTRUCTURE ONLY.

Sec. III-F and Alg. 3 (Update_Col_Jac) of the paper, in numpy float64,
step by step in the paper's notation:
  x_i = ||O_i - C_i||                                            (Eq. dist)
  J_i = (-(O_i - C_i) / x_i)^T Jc_i(q), Jc_i the position Jacobian at C_i (Eq. jac)
  A_ii = activation of the inequality task x_i >= x_M,i with buffer b
  xdot_i = kappa (x* - x_i)                                      (Eq. ref_vel)
  qdot = (J^T A J + V P V^T)^# J^T A A xdot
         + (I - (J^T A J + V P V^T)^# J^T A A J) qdot0           (Eq. task_oriented_solution)
Readings (the design notes list them): the activation is 1 when the sphere
is close (x <= x_M), a raised cosine over the buffer above x_M and 0 beyond
(the printed case split has the two ends swapped); the singular-value
regularisation enters as V P V^T, matching the ||V^T qdot||_P^2 term of the
objective (the printed solution writes V^T P V); P_jj is a raised-cosine
bell of the singular value s_j of J^T A J, reg_max at 0 and zero from
reg_width on; (.)^# is the pseudo-inverse with eigenvalues <= pinv_tol
dropped.  Unlike the library, the eigen-decompositions use numpy.linalg.eigh.
"""
from __future__ import annotations

import numpy as np


def activation(x, x_m, b):
    """A_ii for distances x (array), thresholds x_m and buffer b."""
    x = np.asarray(x, np.float64)
    x_m = np.broadcast_to(np.asarray(x_m, np.float64), x.shape)
    a = 0.5 * (np.cos((x - x_m) * np.pi / b) + 1.0)
    return np.where(x <= x_m, 1.0, np.where(x >= x_m + b, 0.0, a))


def task_jacobian(axes, origins, count, C, O):
    """(x [m], J [m, n]): task variables and task Jacobians (Eqs. dist, jac)."""
    axes = np.asarray(axes, np.float64)
    origins = np.asarray(origins, np.float64)
    C = np.asarray(C, np.float64).reshape(-1, 3)
    O = np.asarray(O, np.float64).reshape(-1, 3)
    m, n = C.shape[0], axes.shape[0]
    d = O - C
    x = np.linalg.norm(d, axis=1)
    J = np.zeros((m, n))
    for i in range(m):
        if x[i] == 0.0:
            continue
        u = -d[i] / x[i]
        for j in range(int(count[i])):
            J[i, j] = u @ np.cross(axes[j], C[i] - origins[j])
    return x, J


def pinv_sym(M, tol):
    w, U = np.linalg.eigh(M)
    inv = np.where(w > tol, 1.0 / np.where(w > tol, w, 1.0), 0.0)
    return (U * inv) @ U.T


def step(axes, origins, count, C, O, x_m, qdot0=None, buffer=0.02, target_offset=0.05, gain=2.0,
         reg_max=1e-3, reg_width=1e-2, pinv_tol=1e-12):
    """One control step: (qdot [n], A [m], x [m])."""
    x, J = task_jacobian(axes, origins, count, C, O)
    n = J.shape[1]
    A = activation(x, x_m, buffer)
    xdot = gain * (np.asarray(x_m, np.float64) + target_offset - x)
    M0 = J.T @ np.diag(A) @ J
    s, V = np.linalg.eigh(M0)
    s = np.abs(s)
    p = np.where(s < reg_width, reg_max * 0.5 * (np.cos(np.pi * s / reg_width) + 1.0), 0.0)
    M = M0 + (V * p) @ V.T
    Minv = pinv_sym(M, pinv_tol)
    AA = np.diag(A * A)
    q0 = np.zeros(n) if qdot0 is None else np.asarray(qdot0, np.float64)
    qdot = Minv @ J.T @ AA @ xdot + (np.eye(n) - Minv @ J.T @ AA @ J) @ q0
    return qdot, A, x
