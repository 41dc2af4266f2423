// Task-priority collision-avoidance controller (Sec. III-F, Alg. 3): host
// code only, the consumer of the sphere queries.  The mathematics is stated
// in include/controller.h; symmetric eigen-decompositions use cyclic Jacobi
// rotations (n <= 16), so the step is deterministic and self-contained.
#include <cmath>
#include <cstring>

#include "common.h"
#include "controller.h"

namespace edtmi {
namespace {

constexpr double PI = 3.14159265358979323846;

// Symmetric a[n][n] -> eigenvalues w[n] and eigenvectors as the columns of
// v[n][n]; a is destroyed.
void jacobi_eigen(int n, double* a, double* w, double* v)
{
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) v[i * n + j] = i == j ? 1.0 : 0.0;
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0.0, tot = 0.0;
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                tot += a[i * n + j] * a[i * n + j];
                if (i != j) off += a[i * n + j] * a[i * n + j];
            }
        if (off <= 1e-30 * tot || off == 0.0) break;
        for (int p = 0; p < n - 1; ++p)
            for (int q = p + 1; q < n; ++q) {
                const double apq = a[p * n + q];
                if (apq == 0.0) continue;
                const double theta = (a[q * n + q] - a[p * n + p]) / (2.0 * apq);
                const double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
                const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
                for (int k = 0; k < n; ++k) {   // columns p, q
                    const double akp = a[k * n + p], akq = a[k * n + q];
                    a[k * n + p] = c * akp - s * akq;
                    a[k * n + q] = s * akp + c * akq;
                }
                for (int k = 0; k < n; ++k) {   // rows p, q
                    const double apk = a[p * n + k], aqk = a[q * n + k];
                    a[p * n + k] = c * apk - s * aqk;
                    a[q * n + k] = s * apk + c * aqk;
                }
                for (int k = 0; k < n; ++k) {
                    const double vkp = v[k * n + p], vkq = v[k * n + q];
                    v[k * n + p] = c * vkp - s * vkq;
                    v[k * n + q] = s * vkp + c * vkq;
                }
            }
    }
    for (int i = 0; i < n; ++i) w[i] = a[i * n + i];
}

double activation(double x, double xm, double b)
{
    if (x <= xm) return 1.0;
    if (x >= xm + b) return 0.0;
    return 0.5 * (std::cos((x - xm) * PI / b) + 1.0);
}

}  // namespace
}  // namespace edtmi

using namespace edtmi;

extern "C" int tp_step(int32_t n, const double* axes, const double* origins, int32_t m,
                       const int32_t* joint_count, const double* centres, const double* nearest,
                       const double* x_min, const double* qdot0, const tp_params_t* p, double* qdot,
                       double* act_out, double* x_out)
{
    if (n < 1 || n > TP_MAX_JOINTS || m < 0 || m > TP_MAX_TASKS || !axes || !origins || !p || !qdot ||
        (m > 0 && (!joint_count || !centres || !nearest || !x_min))) {
        set_error("tp_step: bad sizes or NULL pointer");
        return EDT_ERR_ARG;
    }
    if (!(p->buffer > 0.0) || !(p->gain > 0.0) || !(p->reg_width > 0.0) || !(p->reg_max >= 0.0)) {
        set_error("tp_step: buffer, gain and reg_width must be positive, reg_max non-negative");
        return EDT_ERR_ARG;
    }
    for (int i = 0; i < m; ++i)
        if (joint_count[i] < 0 || joint_count[i] > n) {
            set_error("tp_step: joint_count[%d] = %d outside 0..%d", i, joint_count[i], n);
            return EDT_ERR_ARG;
        }
    double M[TP_MAX_JOINTS * TP_MAX_JOINTS] = {0};    // J^T A J
    double K[TP_MAX_JOINTS * TP_MAX_JOINTS] = {0};    // J^T A A J
    double rhs[TP_MAX_JOINTS] = {0};                  // J^T A A xdot
    for (int i = 0; i < m; ++i) {
        const double* C = centres + 3 * i;
        const double* O = nearest + 3 * i;
        const double d[3] = {O[0] - C[0], O[1] - C[1], O[2] - C[2]};
        const double x = std::sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        const double A = activation(x, x_min[i], p->buffer);
        if (act_out) act_out[i] = A;
        if (x_out) x_out[i] = x;
        if (x == 0.0) continue;   // no direction: the row is zero
        const double u[3] = {-d[0] / x, -d[1] / x, -d[2] / x};
        double J[TP_MAX_JOINTS] = {0};
        for (int j = 0; j < joint_count[i]; ++j) {
            const double* a = axes + 3 * j;
            const double r[3] = {C[0] - origins[3 * j], C[1] - origins[3 * j + 1], C[2] - origins[3 * j + 2]};
            const double cr[3] = {a[1] * r[2] - a[2] * r[1], a[2] * r[0] - a[0] * r[2], a[0] * r[1] - a[1] * r[0]};
            J[j] = u[0] * cr[0] + u[1] * cr[1] + u[2] * cr[2];
        }
        const double xdot = p->gain * (x_min[i] + p->target_offset - x);
        for (int r = 0; r < n; ++r) {
            rhs[r] += A * A * xdot * J[r];
            for (int c = 0; c < n; ++c) {
                M[r * n + c] += A * J[r] * J[c];
                K[r * n + c] += A * A * J[r] * J[c];
            }
        }
    }
    // singular-value regularisation V P V^T from J^T A J = V S V^T
    double E[TP_MAX_JOINTS * TP_MAX_JOINTS], s[TP_MAX_JOINTS], V[TP_MAX_JOINTS * TP_MAX_JOINTS];
    std::memcpy(E, M, sizeof(double) * n * n);
    jacobi_eigen(n, E, s, V);
    double R[TP_MAX_JOINTS * TP_MAX_JOINTS];
    std::memcpy(R, M, sizeof(double) * n * n);
    for (int k = 0; k < n; ++k) {
        const double sk = std::fabs(s[k]);
        const double pk = sk < p->reg_width ? p->reg_max * 0.5 * (std::cos(PI * sk / p->reg_width) + 1.0) : 0.0;
        if (pk == 0.0) continue;
        for (int r = 0; r < n; ++r)
            for (int c = 0; c < n; ++c) R[r * n + c] += pk * V[r * n + k] * V[c * n + k];
    }
    // M^# through the eigen-decomposition of the regularised matrix
    double W[TP_MAX_JOINTS], U[TP_MAX_JOINTS * TP_MAX_JOINTS], Minv[TP_MAX_JOINTS * TP_MAX_JOINTS] = {0};
    std::memcpy(E, R, sizeof(double) * n * n);
    jacobi_eigen(n, E, W, U);
    for (int k = 0; k < n; ++k) {
        if (!(W[k] > p->pinv_tol)) continue;
        const double inv = 1.0 / W[k];
        for (int r = 0; r < n; ++r)
            for (int c = 0; c < n; ++c) Minv[r * n + c] += inv * U[r * n + k] * U[c * n + k];
    }
    // qdot = M^# rhs + (I - M^# K) qdot0
    double MK[TP_MAX_JOINTS * TP_MAX_JOINTS] = {0};
    for (int r = 0; r < n; ++r)
        for (int c = 0; c < n; ++c) {
            double acc = 0.0;
            for (int k = 0; k < n; ++k) acc += Minv[r * n + k] * K[k * n + c];
            MK[r * n + c] = acc;
        }
    for (int r = 0; r < n; ++r) {
        double acc = 0.0;
        for (int k = 0; k < n; ++k) acc += Minv[r * n + k] * rhs[k];
        if (qdot0) {
            for (int k = 0; k < n; ++k) acc += ((r == k ? 1.0 : 0.0) - MK[r * n + k]) * qdot0[k];
        }
        qdot[r] = acc;
    }
    return EDT_OK;
}
