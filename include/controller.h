/*
 * controller.h -- C ABI of the task-priority collision-avoidance controller
 * in libedtmi.so (Sec. III-F and Alg. 3 of arXiv 2407.02363), the consumer
 * of the distance queries (edt_query_spheres).  Host code, float64,
 * synchronous; nothing here touches the GPU.
 *
 * One call is one control step for m scalar avoidance tasks (obstacle and
 * self-collision tasks alike: the caller stacks them).  Task i belongs to a
 * bounding sphere with centre C_i and the closest obstacle point O_i (the
 * query's nearest occupied voxel centre):
 *   x_i   = ||O_i - C_i||                                   (Eq. dist)
 *   J_i   = (-(O_i - C_i) / x_i)^T Jc_i(q)                  (Eq. jac)
 *           where Jc_i is the position Jacobian at C_i of a revolute chain:
 *           column j = a_j x (C_i - p_j) for the joints j < joint_count[i]
 *           that move the sphere, 0 for the others; J_i = 0 when x_i = 0
 *   A_ii  = activation of the inequality task x_i >= x_M,i with transition
 *           buffer b: 1 for x_i <= x_M,i, (cos((x_i - x_M,i) pi / b) + 1) / 2
 *           for x_M,i < x_i < x_M,i + b, 0 beyond (the printed case split
 *           reversed: the task must be active when the sphere is close)
 *   xdot_i = kappa (x*_i - x_i), x*_i = x_M,i + target_offset (Eq. ref_vel)
 * and the joint velocity is the regularised solution (Eq. task_oriented
 * _solution) with singular-value regularisation V P V^T (the objective's
 * ||V^T qdot||_P^2 term) from the eigen-decomposition J^T A J = V S V^T:
 *   M     = J^T A J + V P V^T,  P_jj = reg_max (cos(pi s_j / reg_width) + 1)
 *           / 2 for s_j < reg_width, else 0 (a bell over the singular value)
 *   qdot  = M^# J^T A A xdot + (I - M^# J^T A A J) qdot0
 * M^# is the pseudo-inverse through M's eigen-decomposition, eigenvalues at
 * or below pinv_tol counting as zero.
 */
#ifndef EDTMI_CONTROLLER_H
#define EDTMI_CONTROLLER_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define TP_MAX_JOINTS 16
#define TP_MAX_TASKS 256

typedef struct tp_params_t {
    double buffer;          /* b, metres (the paper uses 0.02 for collision avoidance) */
    double target_offset;   /* x* - x_M, metres, > 0 */
    double gain;            /* kappa, 1/s */
    double reg_max;         /* peak of the singular-value regularisation */
    double reg_width;       /* singular values of J^T A J at or above this are not regularised */
    double pinv_tol;        /* eigenvalues <= pinv_tol count as zero in M^# */
} tp_params_t;

/*
 * tp_step -- one control step.  All pointers are host memory.
 *   axes, origins  double [n_joints][3]: joint axes (unit) and a point on
 *                  each axis, world frame, at the current state
 *   joint_count    int32 [m]: task i is moved by joints 0 .. joint_count[i]-1
 *   centres, nearest  double [m][3]: C_i and O_i, world frame
 *   x_min          double [m]: x_M,i (e.g. sphere radius + safety margin)
 *   qdot0          double [n_joints] (nullable = 0): lower-priority joint velocity
 *   qdot           double [n_joints] out
 *   activation, x  double [m] out (nullable): A_ii and x_i
 * Returns EDT_OK (0) or EDT_ERR_ARG (-1) for sizes outside
 * 1..TP_MAX_JOINTS / 0..TP_MAX_TASKS, NULL pointers, a non-positive
 * buffer, gain or reg_width, or a joint_count outside 0..n_joints.
 */
int tp_step(int32_t n_joints, const double* axes, const double* origins, int32_t m,
            const int32_t* joint_count, const double* centres, const double* nearest,
            const double* x_min, const double* qdot0, const tp_params_t* params, double* qdot,
            double* activation, double* x);

#ifdef __cplusplus
}
#endif
#endif /* EDTMI_CONTROLLER_H */
