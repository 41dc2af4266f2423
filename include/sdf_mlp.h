/*
 * sdf_mlp.h -- C ABI of the learned self-distance surrogate in libedtmi.so.
 *
 * A small MLP maps a joint state q (7 joints) to the distance, in voxels,
 * between each of 12 arm bounding spheres and the self-collision obstacle
 * set -- the task variable x_s of Eq. selftaskvar (Sec. III-E) -- so that
 * most look-ahead states skip the exact self-map EDT.  The paper has no
 * such network: the exact self-map EDT (edt.h) produces its training labels,
 * stays the fallback for every state whose prediction lies within the
 * safety margin plus the network's measured error bound (per sphere, from
 * held-out states: sdf_mlp_calibrate), and is what that error is measured
 * against.
 *
 * Network: input [sin q1, cos q1, ..., sin q7, cos q7] -> 256 -> 256 -> 256
 * -> 12, ReLU between layers.  BF16 inputs, weights and hidden activations
 * (round to nearest even), FP32 accumulation on the matrix cores (MFMA),
 * FP32 biases, FP32 master weights and Adam moments, mean squared error.
 *
 * Parameters live in ONE flat float32 block of SDF_MLP_PARAMS values at the
 * fixed offsets below (weights W[out][in] row-major, the input dimension
 * padded to 32 and the output dimension to 32 with zeros that stay zero),
 * plus a bfloat16 copy of the same block (sdf_mlp_pack / sdf_mlp_adam keep
 * it in step) that the matrix kernels read.  Gradients use the same layout.
 *
 * Conventions as in edt.h: device pointers, caller-owned buffers, stream as
 * void*, nothing allocated, negative status on error.  Any batch >= 1 works:
 * the workspace pads it to a multiple of 64 rows internally.
 */
#ifndef EDTMI_SDF_MLP_H
#define EDTMI_SDF_MLP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SDF_MLP_JOINTS 7
#define SDF_MLP_IN 14
#define SDF_MLP_HIDDEN 256
#define SDF_MLP_OUT 12
#define SDF_MLP_IN_PAD 32
#define SDF_MLP_OUT_PAD 32

enum {
    SDF_MLP_W1 = 0,        /* [256][32]  */
    SDF_MLP_B1 = 8192,     /* [256]      */
    SDF_MLP_W2 = 8448,     /* [256][256] */
    SDF_MLP_B2 = 73984,    /* [256]      */
    SDF_MLP_W3 = 74240,    /* [256][256] */
    SDF_MLP_B3 = 139776,   /* [256]      */
    SDF_MLP_W4 = 140032,   /* [32][256]  */
    SDF_MLP_B4 = 148224,   /* [32]       */
    SDF_MLP_PARAMS = 148256
};

/* Workspace bytes for a batch (encoded inputs, saved activations, outputs,
 * gradients of the backward pass, loss and weight-gradient partial sums). */
size_t sdf_mlp_workspace_bytes(int32_t batch);

/* w16 = bfloat16(master), element by element (round to nearest even). */
int sdf_mlp_pack(const float* master, uint16_t* w16, void* stream);

/*
 * sdf_mlp_forward -- predicted distances for `batch` joint states.
 *   w16     bfloat16 parameter block (weights read from it)
 *   master  float32 parameter block (biases read from it)
 *   q       float32 [n_rows][7] joint angles, radians
 *   idx     int32 [batch] (nullable): row b of the batch is state q[idx[b]]
 *           (a minibatch gathered inside the kernel); NULL = rows 0..batch-1,
 *           which needs n_rows >= batch.  An index outside [0, n_rows)
 *           gives that row NaN inputs (so NaN outputs) instead of a read
 *           outside q.
 *   y       float32 [batch][12] out, voxels (NULL: keep only in ws)
 * Saves the encoded inputs and hidden activations in ws for
 * sdf_mlp_backward.
 */
int sdf_mlp_forward(const uint16_t* w16, const float* master, const float* q, int32_t n_rows,
                    const int32_t* idx, int32_t batch, float* y, void* ws, size_t ws_bytes,
                    void* stream);

/*
 * sdf_mlp_backward -- gradients of the mean squared error of the last
 * sdf_mlp_forward on ws against the targets.
 *   target    float32 [n_rows][12], voxels; row b of the batch uses
 *             target[idx[b]] (idx as in sdf_mlp_forward, the same array).
 *   clip_vox  > 0: every target is first replaced by min(target, clip_vox)
 *             (the network then learns the distance saturated at clip_vox);
 *             <= 0: no clipping.
 *   grad      float32 parameter-block layout, fully overwritten.
 *   loss      float32 device scalar out (nullable): the mean squared error.
 * dY and every masked upstream gradient are rounded to bfloat16 before
 * they enter a matrix product.  Weight and bias gradients reduce over the
 * batch in fixed-size chunks whose partial sums are added in chunk order
 * (no atomics), so two runs give identical bits.
 */
int sdf_mlp_backward(const uint16_t* w16, const float* target, int32_t n_rows, const int32_t* idx,
                     int32_t batch, float clip_vox, float* grad, float* loss, void* ws,
                     size_t ws_bytes, void* stream);

/*
 * sdf_mlp_adam -- one Adam step (bias-corrected; step counts from 1) on
 * the float32 master block with moments m, v (same layout, start at zero),
 * then refresh the bfloat16 copy w16.
 */
int sdf_mlp_adam(float* master, uint16_t* w16, float* m, float* v, const float* grad,
                 int32_t step, float lr, float beta1, float beta2, float eps, void* stream);

/*
 * sdf_mlp_fallback -- the exact-EDT fallback rule.  State b needs the exact
 * self-map transform when some sphere i has predicted clearance
 * y[b][i] * voxel - radii[i] below margin + eps_vox[i] * voxel (metres),
 * i.e. within the safety margin once the surrogate's error bound for that
 * sphere is allowed for; a NaN prediction always needs it.  Evaluated in
 * float32 in exactly that order: c = y * voxel - r, t = margin +
 * eps * voxel, exact iff !(c >= t).
 *   radii, eps_vox  float32 [12] device arrays (metres, voxels).
 *   need   int32 [batch] out: 1 = run the exact EDT for this state.
 *   count  int32 device scalar out: number of such states.
 */
int sdf_mlp_fallback(const float* y, const float* radii, const float* eps_vox, int32_t batch,
                     float voxel, float margin, int32_t* need, int32_t* count, void* stream);

/*
 * sdf_mlp_infer -- sdf_mlp_forward for inference: the same predictions, bit
 * for bit, in one launch (one work-group per 64 states, the activations kept
 * on chip), with no workspace and nothing kept for a backward pass.
 *   q     float32 [batch][7] joint angles, radians, device.
 *   y     float32 [batch][12] out, voxels, device.
 *   need  int32 [batch] out (nullable): when given, the fallback rule of
 *         sdf_mlp_fallback is applied to y with radii, eps_vox, voxel and
 *         margin (same arguments, same float32 evaluation, same decisions);
 *         its count is not produced.  radii and eps_vox may be NULL when
 *         need is.
 */
int sdf_mlp_infer(const uint16_t* w16, const float* master, const float* q, int32_t batch, float* y,
                  const float* radii, const float* eps_vox, float voxel, float margin, int32_t* need,
                  void* stream);

/*
 * sdf_mlp_select -- the distances a look-ahead batch ends with: the exact
 * ones for the states that needed the exact self-map transform, the
 * predictions for the rest.  For every state b and sphere i:
 *   out[b][i] = need[b] != 0 ? exact[b * exact_row + i * exact_col] : y[b][i]
 *   y, out   float32 [batch][12] device, voxels (out may be y).
 *   need     int32 [batch] device: sdf_mlp_fallback's output.
 *   exact    float32 device, strided by exact_row / exact_col floats, so the
 *            dist_vox word of edt_sphere_result_t records can be read in
 *            place (records [batch][12] of 16 words: exact = &rec->dist_vox,
 *            exact_row = 192, exact_col = 16).  Rows with need[b] == 0 are
 *            not read.
 * A selection, no arithmetic: the copied values keep their bits.
 */
int sdf_mlp_select(const float* y, const int32_t* need, const float* exact, int32_t exact_row,
                   int32_t exact_col, int32_t batch, float* out, void* stream);

/*
 * sdf_mlp_calibrate -- the error bound the fallback rule allows for, from
 * held-out states with exact labels.  For every sphere i:
 *   eps_vox[i] = max(0, max over rows b with target[b][i] < clip_vox of
 *                pred[b][i] - target[b][i])        (float32 difference)
 * i.e. the largest overestimate of the distance on the held-out rows whose
 * exact distance lies below the clip (clip_vox <= 0: every row).  Only an
 * overestimate can hide a sphere inside the margin, and a sphere inside the
 * margin has an exact distance below the clip as long as
 * (margin + radius) / voxel + eps < clip_vox.  A NaN prediction makes the
 * bound +inf.
 *   pred, target  float32 [batch][12] device (voxels); eps_vox float32 [12]
 *   device out, fully overwritten.
 */
int sdf_mlp_calibrate(const float* pred, const float* target, int32_t batch, float clip_vox,
                      float* eps_vox, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* EDTMI_SDF_MLP_H */
