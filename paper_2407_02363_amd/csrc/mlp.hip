// Learned self-distance surrogate: BF16 MFMA kernels for the forward pass,
// the backward pass and Adam, plus the exact-EDT fallback rule.
//
// Every matrix product is one kernel, k_gemm: a 64 x 64 tile per 256-thread
// work-group, 32 x 32 per wave as 2 x 2 blocks of v_mfma_f32_16x16x32_bf16,
// fed straight from global memory (all operands are L2-resident: at most
// 4096 x 256 bf16).  Lane l of an MFMA holds A[l % 16][8 (l / 16) + i],
// B[8 (l / 16) + i][l % 16] and C[4 (l / 16) + i][l % 16].  The epilogue
// decides what a product becomes:
//   HID  hidden layer:  bf16(relu(acc + bias)), relu(NaN) = NaN
//   OUT  output layer:  acc + bias (float32)
//   DX   upstream gradient: bf16(acc masked where the layer input h > 0)
// Weight gradients (a reduction over the batch) have their own kernel,
// k_gemm_dw: the batch is cut into KS chunks, every (64 x 64 tile, chunk)
// work-group stages its operands through LDS transposed, writes an FP32
// partial tile (and the bias partial sums), and k_reduce_dw adds the KS
// partials in chunk order, so two runs give identical bits.
#include "common.h"
#include "sdf_mlp.h"

namespace edtmi {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int HID = SDF_MLP_HIDDEN;
constexpr int INP = SDF_MLP_IN_PAD;
constexpr int OUTP = SDF_MLP_OUT_PAD;
constexpr int ROW_ALIGN = 64;

__host__ __device__ inline int padded_rows(int b) { return (b + ROW_ALIGN - 1) / ROW_ALIGN * ROW_ALIGN; }

// float -> bfloat16 bits, round to nearest even (NaN -> quiet NaN)
__device__ __forceinline__ uint16_t f2bf(float f)
{
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7FFFFFFFu) > 0x7F800000u) return 0x7FC0u;
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// Workspace layout (bytes) for padded batch P.
struct WsLayout {
    size_t x, h1, h2, h3, y, dy, dpa, dpb, part, dwpart, dbpart, total;
};

// batch chunks of the weight-gradient reduction: the largest of 16, 8, 4,
// 2, 1 that cuts the P / 32 MFMA steps evenly
__host__ __device__ inline int dw_chunks(int P)
{
    const int steps = P / 32;
    int ks = 16;
    while (steps % ks) ks >>= 1;
    return ks;
}

__host__ __device__ inline WsLayout ws_layout(int P)
{
    WsLayout w;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t at = o;
        o += (bytes + 255) / 256 * 256;
        return at;
    };
    w.x = take((size_t)P * INP * 2);
    w.h1 = take((size_t)P * HID * 2);
    w.h2 = take((size_t)P * HID * 2);
    w.h3 = take((size_t)P * HID * 2);
    w.y = take((size_t)P * OUTP * 4);
    w.dy = take((size_t)P * OUTP * 2);
    w.dpa = take((size_t)P * HID * 2);
    w.dpb = take((size_t)P * HID * 2);
    w.part = take(1024 * 4);
    w.dwpart = take((size_t)dw_chunks(P) * HID * HID * 4);
    w.dbpart = take((size_t)dw_chunks(P) * HID * 4);
    w.total = o;
    return w;
}

enum { EPI_HID = 0, EPI_OUT = 1, EPI_DX = 2 };

struct GemmArgs {
    const uint16_t* A;
    int lda;
    const uint16_t* B;
    int ldb;
    int M, N, K;           // K is a multiple of 32
    const float* bias;     // HID / OUT
    const uint16_t* mask;  // DX: layer input h, [M][ldm]
    int ldm;
    uint16_t* out16;       // HID / DX
    float* out32;          // OUT / DW
    int ldo;
};

// C[m][n] = sum_k A(m, k) B(k, n) with A(m, k) = TA ? A[k][m] : A[m][k] and
// B(k, n) = TB ? B[n][k] : B[k][n].
template <bool TA, bool TB, int EPI>
__global__ __launch_bounds__(256) void k_gemm(GemmArgs g)
{
    const int wave = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    const int m0 = blockIdx.y * 64 + (wave >> 1) * 32;
    const int n0 = blockIdx.x * 64 + (wave & 1) * 32;
    const int r = lane & 15;
    const int kq = (lane >> 4) * 8;
    f32x4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};

    for (int k0 = 0; k0 < g.K; k0 += 32) {
        const int k = k0 + kq;
        bf16x8 a[2], b[2];
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            const int m = m0 + 16 * i + r;
            if (m < g.M) {
                if constexpr (!TA) {
                    const uint4 v = *reinterpret_cast<const uint4*>(g.A + (size_t)m * g.lda + k);
                    a[i] = __builtin_bit_cast(bf16x8, v);
                } else {
#pragma unroll
                    for (int e = 0; e < 8; ++e)
                        a[i][e] = __builtin_bit_cast(__bf16, g.A[(size_t)(k + e) * g.lda + m]);
                }
            } else {
                a[i] = __builtin_bit_cast(bf16x8, make_uint4(0, 0, 0, 0));
            }
        }
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int n = n0 + 16 * j + r;
            if (n < g.N) {
                if constexpr (TB) {
                    const uint4 v = *reinterpret_cast<const uint4*>(g.B + (size_t)n * g.ldb + k);
                    b[j] = __builtin_bit_cast(bf16x8, v);
                } else {
#pragma unroll
                    for (int e = 0; e < 8; ++e)
                        b[j][e] = __builtin_bit_cast(__bf16, g.B[(size_t)(k + e) * g.ldb + n]);
                }
            } else {
                b[j] = __builtin_bit_cast(bf16x8, make_uint4(0, 0, 0, 0));
            }
        }
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j)
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
    }

#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int m = m0 + 16 * i + 4 * (lane >> 4) + e;
                const int n = n0 + 16 * j + r;
                if (m >= g.M || n >= g.N) continue;
                const float v = acc[i][j][e];
                if constexpr (EPI == EPI_HID) {
                    const float z = v + g.bias[n];
                    // ReLU that keeps a NaN (a poisoned row stays visible)
                    g.out16[(size_t)m * g.ldo + n] = f2bf((z > 0.0f || z != z) ? z : 0.0f);
                } else if constexpr (EPI == EPI_OUT) {
                    g.out32[(size_t)m * g.ldo + n] = v + g.bias[n];
                } else {
                    const bool on = bf2f(g.mask[(size_t)m * g.ldm + n]) > 0.0f;
                    g.out16[(size_t)m * g.ldo + n] = f2bf(on ? v : 0.0f);
                }
            }
}

// Weight-gradient partials.  dW[m][n] = sum_b up[b][m] act[b][n] over the
// batch rows b of chunk blockIdx.z; M = outputs (rows of up), N = inputs.
// Both operands arrive as coalesced 16-byte loads of 32 batch rows and are
// stored transposed in LDS ([m][k] and [n][k], rows padded to 40 elements),
// so every MFMA operand is one 16-byte LDS read.  The work-groups of the
// first column of tiles also sum up over their rows (the bias gradient).
constexpr int DW_LDK = 40;

__global__ __launch_bounds__(256) void k_gemm_dw(const uint16_t* __restrict__ up, int M,
                                                 const uint16_t* __restrict__ act, int N, int KC,
                                                 float* __restrict__ dwpart, float* __restrict__ dbpart)
{
    __shared__ __attribute__((aligned(16))) uint16_t sA[64 * DW_LDK];
    __shared__ __attribute__((aligned(16))) uint16_t sB[64 * DW_LDK];
    const int t = threadIdx.x;
    const int wave = t >> 6;
    const int lane = t & 63;
    const int m0 = blockIdx.y * 64, n0 = blockIdx.x * 64;
    const int s = blockIdx.z;
    const int mw = (wave >> 1) * 32, nw = (wave & 1) * 32;
    const int r = lane & 15;
    const int kq = (lane >> 4) * 8;
    // loader: row kr of the 32-row step, 8 columns from c8
    const int kr = t >> 3, c8 = (t & 7) * 8;
    const bool bias = blockIdx.x == 0;
    float bsum = 0.0f;
    f32x4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};

    const int kbeg = s * KC;
    for (int k0 = kbeg; k0 < kbeg + KC; k0 += 32) {
        uint4 va = make_uint4(0, 0, 0, 0), vb = make_uint4(0, 0, 0, 0);
        if (m0 + c8 < M) va = *reinterpret_cast<const uint4*>(up + (size_t)(k0 + kr) * M + m0 + c8);
        if (n0 + c8 < N) vb = *reinterpret_cast<const uint4*>(act + (size_t)(k0 + kr) * N + n0 + c8);
        const uint16_t* ea = reinterpret_cast<const uint16_t*>(&va);
        const uint16_t* eb = reinterpret_cast<const uint16_t*>(&vb);
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            sA[(c8 + e) * DW_LDK + kr] = ea[e];
            sB[(c8 + e) * DW_LDK + kr] = eb[e];
        }
        __syncthreads();
        bf16x8 a[2], b[2];
#pragma unroll
        for (int i = 0; i < 2; ++i)
            a[i] = *reinterpret_cast<const bf16x8*>(sA + (mw + 16 * i + r) * DW_LDK + kq);
#pragma unroll
        for (int j = 0; j < 2; ++j)
            b[j] = *reinterpret_cast<const bf16x8*>(sB + (nw + 16 * j + r) * DW_LDK + kq);
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j)
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
        if (bias && t < 64) {
#pragma unroll 8
            for (int k = 0; k < 32; ++k) bsum += bf2f(sA[t * DW_LDK + k]);
        }
        __syncthreads();
    }
    float* out = dwpart + (size_t)s * M * N;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int m = m0 + mw + 16 * i + 4 * (lane >> 4) + e;
                const int n = n0 + nw + 16 * j + r;
                if (m < M && n < N) out[(size_t)m * N + n] = acc[i][j][e];
            }
    if (bias && t < 64 && m0 + t < M) dbpart[(size_t)s * M + m0 + t] = bsum;
}

// grad[m][n] = sum over chunks s = 0 .. KS-1 of the partials, in that order
__global__ void k_reduce_dw(const float* __restrict__ dwpart, const float* __restrict__ dbpart, int M,
                            int N, int KS, float* __restrict__ gw, float* __restrict__ gb)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int MN = M * N;
    if (i < MN) {
        float a = 0.0f;
        for (int s = 0; s < KS; ++s) a += dwpart[(size_t)s * MN + i];
        gw[i] = a;
    } else if (i < MN + M) {
        const int m = i - MN;
        float a = 0.0f;
        for (int s = 0; s < KS; ++s) a += dbpart[(size_t)s * M + m];
        gb[m] = a;
    }
}

// x = [sin q1, cos q1, ..., sin q7, cos q7, 0 ...] in bf16 for state
// idx[b] (b if idx is NULL); padded rows 0; NaN for an index outside
// [0, n_rows)
__global__ void k_encode(const float* __restrict__ q, int n_rows, const int* __restrict__ idx,
                         int batch, int P, uint16_t* __restrict__ x)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= P * INP) return;
    const int b = i / INP, c = i % INP;
    float v = 0.0f;
    if (b < batch && c < 2 * SDF_MLP_JOINTS) {
        const int row = idx ? idx[b] : b;
        if (row >= 0 && row < n_rows) {
            const float a = q[(size_t)row * SDF_MLP_JOINTS + (c >> 1)];
            v = (c & 1) ? cosf(a) : sinf(a);
        } else {
            v = __builtin_nanf("");   // an index outside q poisons its row
        }
    }
    x[i] = f2bf(v);
}

// The whole forward pass for inference, one 512-thread work-group per 64
// rows of the batch: the encoded input and the hidden activations stay in
// LDS (row stride HID + 8 bf16) and the weights come from L2.  Wave w owns
// the output columns [32 w, 32 w + 32) of a layer; it loads its weight rows
// for every K step at once and then runs its products, only over the 16-row
// tiles that hold states.  Every product is the same sequence of
// v_mfma_f32_16x16x32_bf16 over K in steps of 32 as in k_gemm, with the same
// epilogues, so y is bit-identical to sdf_mlp_forward's.  With need given,
// the work-group also applies k_fallback's rule to its rows.
constexpr int INF_LD = HID + 8;

__global__ __launch_bounds__(512) void k_mlp_infer(const uint16_t* __restrict__ w16,
                                                   const float* __restrict__ master,
                                                   const float* __restrict__ q, int batch,
                                                   float* __restrict__ y, const float* __restrict__ radii,
                                                   const float* __restrict__ eps, float voxel, float margin,
                                                   int* __restrict__ need)
{
    __shared__ __attribute__((aligned(16))) uint16_t act[2][64 * INF_LD];
    __shared__ float yout[64 * SDF_MLP_OUT];
    const int t = threadIdx.x;
    const int wave = t >> 6;
    const int lane = t & 63;
    const int row0 = blockIdx.x * 64;
    const int rows = min(64, batch - row0);
    const int mt = (rows + 15) >> 4;   // 16-row tiles that hold states
    // encode: [sin q1, cos q1, ..., sin q7, cos q7, 0 ...] as bf16 (k_encode's values)
    for (int i = t; i < 64 * INP; i += 512) {
        const int b = i / INP, c = i % INP;
        float v = 0.0f;
        if (b < rows && c < 2 * SDF_MLP_JOINTS) {
            const float a = q[(size_t)(row0 + b) * SDF_MLP_JOINTS + (c >> 1)];
            v = (c & 1) ? cosf(a) : sinf(a);
        }
        act[0][b * INF_LD + c] = f2bf(v);
    }
    __syncthreads();
    const int r = lane & 15;
    const int kq = (lane >> 4) * 8;
#pragma unroll
    for (int l = 0; l < 4; ++l) {
        const uint16_t* A = act[l & 1];
        uint16_t* O = act[(l & 1) ^ 1];
        constexpr int KS_MAX = HID / 32;
        const int K = l == 0 ? INP : HID;
        const int N = l == 3 ? OUTP : HID;
        const uint16_t* W = w16 + (l == 0 ? SDF_MLP_W1 : l == 1 ? SDF_MLP_W2 : l == 2 ? SDF_MLP_W3 : SDF_MLP_W4);
        const float* bias = master + (l == 0 ? SDF_MLP_B1 : l == 1 ? SDF_MLP_B2 : l == 2 ? SDF_MLP_B3 : SDF_MLP_B4);
        const int n0 = wave * 32;
        if (n0 < N) {
            bf16x8 b[2][KS_MAX];
#pragma unroll
            for (int ks = 0; ks < KS_MAX; ++ks)
#pragma unroll
                for (int j = 0; j < 2; ++j)
                    if (ks * 32 < K)
                        b[j][ks] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(
                                                                  W + (size_t)(n0 + 16 * j + r) * K + ks * 32 + kq));
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                if (i >= mt) break;
                f32x4 acc[2] = {f32x4{0.0f, 0.0f, 0.0f, 0.0f}, f32x4{0.0f, 0.0f, 0.0f, 0.0f}};
#pragma unroll
                for (int ks = 0; ks < KS_MAX; ++ks) {
                    if (ks * 32 >= K) break;
                    const bf16x8 a = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(
                                                                    A + (16 * i + r) * INF_LD + ks * 32 + kq));
#pragma unroll
                    for (int j = 0; j < 2; ++j)
                        acc[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b[j][ks], acc[j], 0, 0, 0);
                }
#pragma unroll
                for (int j = 0; j < 2; ++j)
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const int m = 16 * i + 4 * (lane >> 4) + e;
                        const int n = n0 + 16 * j + r;
                        const float z = acc[j][e] + bias[n];
                        if (l < 3) {
                            O[m * INF_LD + n] = f2bf((z > 0.0f || z != z) ? z : 0.0f);
                        } else if (n < SDF_MLP_OUT && m < rows) {
                            y[(size_t)(row0 + m) * SDF_MLP_OUT + n] = z;
                            yout[m * SDF_MLP_OUT + n] = z;
                        }
                    }
            }
        }
        __syncthreads();
    }
    if (need && t < rows) {
        int flag = 0;
        for (int i = 0; i < SDF_MLP_OUT; ++i) {
            const float c = yout[t * SDF_MLP_OUT + i] * voxel - radii[i];
            const float thresh = margin + eps[i] * voxel;
            if (!(c >= thresh)) flag = 1;   // NaN predictions also fall back
        }
        need[row0 + t] = flag;
    }
}

// y32 [P][32] -> y [batch][12]
__global__ void k_copy_out(const float* __restrict__ y32, int batch, float* __restrict__ y)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= batch * SDF_MLP_OUT) return;
    y[i] = y32[(i / SDF_MLP_OUT) * OUTP + i % SDF_MLP_OUT];
}

// dY = bf16(2 (y - t) / (batch * 12)) on valid entries, 0 elsewhere, with
// t = min(target[idx[b]], clip) (clip <= 0: no clipping; NaN for an index
// outside [0, n_rows)); block partial
// sums of (y - t)^2 in a fixed order
__global__ __launch_bounds__(256) void k_loss_dy(const float* __restrict__ y32,
                                                 const float* __restrict__ target, int n_rows,
                                                 const int* __restrict__ idx, float clip, int batch,
                                                 int P, uint16_t* __restrict__ dy,
                                                 float* __restrict__ part)
{
    __shared__ float red[256];
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const float scale = 2.0f / (float)(batch * SDF_MLP_OUT);
    float sq = 0.0f;
    if (i < P * OUTP) {
        const int b = i / OUTP, c = i % OUTP;
        float g = 0.0f;
        if (b < batch && c < SDF_MLP_OUT) {
            const int row = idx ? idx[b] : b;
            float t = __builtin_nanf("");   // an index outside target poisons its row
            if (row >= 0 && row < n_rows) t = target[(size_t)row * SDF_MLP_OUT + c];
            if (clip > 0.0f && t > clip) t = clip;
            const float d = y32[i] - t;
            sq = d * d;
            g = d * scale;
        }
        dy[i] = f2bf(g);
    }
    red[threadIdx.x] = sq;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(256) void k_loss_final(const float* __restrict__ part, int nparts,
                                                    int batch, float* __restrict__ loss)
{
    __shared__ float red[256];
    float s = 0.0f;
    for (int i = threadIdx.x; i < nparts; i += 256) s += part[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) *loss = red[0] / (float)(batch * SDF_MLP_OUT);
}

__global__ void k_pack(const float* __restrict__ master, uint16_t* __restrict__ w16, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) w16[i] = f2bf(master[i]);
}

__global__ void k_adam(float* __restrict__ w, uint16_t* __restrict__ w16, float* __restrict__ m,
                       float* __restrict__ v, const float* __restrict__ g, int n, float lr, float b1,
                       float b2, float eps, float c1, float c2)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float wi = w[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    w[i] = wi;
    w16[i] = f2bf(wi);
}

__global__ __launch_bounds__(256) void k_fallback(const float* __restrict__ y,
                                                  const float* __restrict__ radii,
                                                  const float* __restrict__ eps, int batch,
                                                  float voxel, float margin, int* __restrict__ need,
                                                  int* __restrict__ count)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    int flag = 0;
    if (b < batch) {
        for (int i = 0; i < SDF_MLP_OUT; ++i) {
            const float c = y[b * SDF_MLP_OUT + i] * voxel - radii[i];
            const float thresh = margin + eps[i] * voxel;
            if (!(c >= thresh)) flag = 1;   // NaN predictions also fall back
        }
        need[b] = flag;
    }
    const unsigned long long bal = __ballot(flag);
    if ((threadIdx.x & 63) == 0 && bal) atomicAdd(count, (int)__popcll(bal));
}

// out[b][i] = need[b] ? exact[b * erow + i * ecol] : y[b][i]
__global__ void k_select(const float* __restrict__ y, const int* __restrict__ need,
                         const float* __restrict__ exact, int erow, int ecol, int batch,
                         float* __restrict__ out)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= batch * SDF_MLP_OUT) return;
    const int b = k / SDF_MLP_OUT, i = k % SDF_MLP_OUT;
    out[k] = need[b] ? exact[(size_t)b * erow + (size_t)i * ecol] : y[k];
}

__global__ void k_zero_int(int* p) { *p = 0; }

__global__ void k_zero_f32(float* p, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.0f;
}

// eps[i] = max(0, max over rows b with target[b][i] < clip of
// pred[b][i] - target[b][i]) (clip <= 0: every row); a NaN prediction
// gives +inf.  Non-negative floats order like their bit patterns, so the
// maximum is an integer atomicMax on the bits and independent of order.
__global__ __launch_bounds__(256) void k_calibrate(const float* __restrict__ pred,
                                                   const float* __restrict__ target, int batch,
                                                   float clip, unsigned* __restrict__ eps)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= batch * SDF_MLP_OUT) return;
    const float t = target[i], p = pred[i];
    if (clip > 0.0f && !(t < clip)) return;
    float d = p - t;
    if (p != p) d = __builtin_huge_valf();
    if (d > 0.0f) atomicMax(eps + i % SDF_MLP_OUT, __float_as_uint(d));
}

template <bool TA, bool TB, int EPI>
int gemm(const GemmArgs& a, hipStream_t st)
{
    if (a.K % 32) {
        set_error("k_gemm: K=%d is not a multiple of 32", a.K);
        return EDT_ERR_ARG;
    }
    const dim3 grid((a.N + 63) / 64, (a.M + 63) / 64);
    hipLaunchKernelGGL((k_gemm<TA, TB, EPI>), grid, dim3(256), 0, st, a);
    return check_launch("k_gemm");
}

GemmArgs args0()
{
    GemmArgs a{};
    return a;
}

}  // namespace

}  // namespace edtmi

using namespace edtmi;

extern "C" {

size_t sdf_mlp_workspace_bytes(int32_t batch)
{
    if (batch < 1) return 0;
    return ws_layout(padded_rows(batch)).total;
}

int sdf_mlp_pack(const float* master, uint16_t* w16, void* stream)
{
    if (!master || !w16) {
        set_error("sdf_mlp_pack: NULL pointer");
        return EDT_ERR_ARG;
    }
    hipLaunchKernelGGL(k_pack, dim3((SDF_MLP_PARAMS + 255) / 256), dim3(256), 0, as_stream(stream),
                       master, w16, (int)SDF_MLP_PARAMS);
    return check_launch("k_pack");
}

int sdf_mlp_forward(const uint16_t* w16, const float* master, const float* q, int32_t n_rows,
                    const int32_t* idx, int32_t batch, float* y, void* ws, size_t ws_bytes,
                    void* stream)
{
    if (!w16 || !master || !q || !ws || batch < 1 || n_rows < 1 || (!idx && n_rows < batch)) {
        set_error("sdf_mlp_forward: NULL pointer, batch < 1, or fewer rows than the batch");
        return EDT_ERR_ARG;
    }
    const int P = padded_rows(batch);
    const WsLayout L = ws_layout(P);
    if (ws_bytes < L.total) {
        set_error("sdf_mlp_forward: workspace %zu < %zu bytes", ws_bytes, L.total);
        return EDT_ERR_WORKSPACE;
    }
    char* w = static_cast<char*>(ws);
    uint16_t* x = reinterpret_cast<uint16_t*>(w + L.x);
    uint16_t* h[3] = {reinterpret_cast<uint16_t*>(w + L.h1), reinterpret_cast<uint16_t*>(w + L.h2),
                      reinterpret_cast<uint16_t*>(w + L.h3)};
    float* y32 = reinterpret_cast<float*>(w + L.y);
    const hipStream_t st = as_stream(stream);
    hipLaunchKernelGGL(k_encode, dim3((P * INP + 255) / 256), dim3(256), 0, st, q, (int)n_rows, idx,
                       (int)batch, P, x);
    int rc = check_launch("k_encode");
    if (rc) return rc;
    const int woff[4] = {SDF_MLP_W1, SDF_MLP_W2, SDF_MLP_W3, SDF_MLP_W4};
    const int boff[4] = {SDF_MLP_B1, SDF_MLP_B2, SDF_MLP_B3, SDF_MLP_B4};
    const uint16_t* in = x;
    int kin = INP;
    for (int l = 0; l < 4; ++l) {
        GemmArgs a = args0();
        a.A = in;
        a.lda = kin;
        a.B = w16 + woff[l];
        a.ldb = kin;
        a.M = P;
        a.K = kin;
        a.bias = master + boff[l];
        if (l < 3) {
            a.N = HID;
            a.out16 = h[l];
            a.ldo = HID;
            rc = gemm<false, true, EPI_HID>(a, st);
            in = h[l];
            kin = HID;
        } else {
            a.N = OUTP;
            a.out32 = y32;
            a.ldo = OUTP;
            rc = gemm<false, true, EPI_OUT>(a, st);
        }
        if (rc) return rc;
    }
    if (y) {
        hipLaunchKernelGGL(k_copy_out, dim3((batch * SDF_MLP_OUT + 255) / 256), dim3(256), 0, st, y32,
                           (int)batch, y);
        rc = check_launch("k_copy_out");
    }
    return rc;
}

int sdf_mlp_backward(const uint16_t* w16, const float* target, int32_t n_rows, const int32_t* idx,
                     int32_t batch, float clip_vox, float* grad, float* loss, void* ws, size_t ws_bytes,
                     void* stream)
{
    if (!w16 || !target || !grad || !ws || batch < 1 || n_rows < 1 || (!idx && n_rows < batch)) {
        set_error("sdf_mlp_backward: NULL pointer, batch < 1, or fewer rows than the batch");
        return EDT_ERR_ARG;
    }
    const int P = padded_rows(batch);
    const WsLayout L = ws_layout(P);
    if (ws_bytes < L.total) {
        set_error("sdf_mlp_backward: workspace %zu < %zu bytes", ws_bytes, L.total);
        return EDT_ERR_WORKSPACE;
    }
    char* w = static_cast<char*>(ws);
    const uint16_t* act[4] = {reinterpret_cast<uint16_t*>(w + L.x), reinterpret_cast<uint16_t*>(w + L.h1),
                              reinterpret_cast<uint16_t*>(w + L.h2), reinterpret_cast<uint16_t*>(w + L.h3)};
    const float* y32 = reinterpret_cast<float*>(w + L.y);
    uint16_t* dy = reinterpret_cast<uint16_t*>(w + L.dy);
    uint16_t* dp[2] = {reinterpret_cast<uint16_t*>(w + L.dpa), reinterpret_cast<uint16_t*>(w + L.dpb)};
    float* part = reinterpret_cast<float*>(w + L.part);
    float* dwpart = reinterpret_cast<float*>(w + L.dwpart);
    float* dbpart = reinterpret_cast<float*>(w + L.dbpart);
    const int KS = dw_chunks(P);
    const hipStream_t st = as_stream(stream);
    const int nblk = (P * OUTP + 255) / 256;
    if (nblk > 1024) {
        set_error("sdf_mlp_backward: batch too large for the loss reduction");
        return EDT_ERR_UNSUPPORTED;
    }
    hipLaunchKernelGGL(k_loss_dy, dim3(nblk), dim3(256), 0, st, y32, target, (int)n_rows, idx,
                       clip_vox, (int)batch, P, dy, part);
    int rc = check_launch("k_loss_dy");
    if (rc) return rc;
    if (loss) {
        hipLaunchKernelGGL(k_loss_final, dim3(1), dim3(256), 0, st, part, nblk, (int)batch, loss);
        if ((rc = check_launch("k_loss_final"))) return rc;
    }
    const int woff[4] = {SDF_MLP_W1, SDF_MLP_W2, SDF_MLP_W3, SDF_MLP_W4};
    const int boff[4] = {SDF_MLP_B1, SDF_MLP_B2, SDF_MLP_B3, SDF_MLP_B4};
    const int nout[4] = {HID, HID, HID, OUTP};
    const int nin[4] = {INP, HID, HID, HID};
    const uint16_t* up = dy;   // upstream gradient of layer l's output, [P][nout]
    for (int l = 3; l >= 0; --l) {
        // dW_l = up^T act_l and db_l = column sums of up: M = nout, N = nin,
        // reduced over the P rows of the batch in KS chunks
        const dim3 g((nin[l] + 63) / 64, (nout[l] + 63) / 64, KS);
        hipLaunchKernelGGL(k_gemm_dw, g, dim3(256), 0, st, up, nout[l], act[l], nin[l], P / KS, dwpart,
                           dbpart);
        if ((rc = check_launch("k_gemm_dw"))) return rc;
        const int nred = nout[l] * nin[l] + nout[l];
        hipLaunchKernelGGL(k_reduce_dw, dim3((nred + 255) / 256), dim3(256), 0, st, dwpart, dbpart,
                           nout[l], nin[l], KS, grad + woff[l], grad + boff[l]);
        if ((rc = check_launch("k_reduce_dw"))) return rc;
        if (l == 0) break;
        // upstream of layer l-1: (up W_l) masked where act_l > 0
        GemmArgs d = args0();
        d.A = up;
        d.lda = nout[l];
        d.B = w16 + woff[l];
        d.ldb = nin[l];
        d.M = P;
        d.N = nin[l];
        d.K = nout[l];
        d.mask = act[l];
        d.ldm = nin[l];
        d.out16 = dp[l & 1];
        d.ldo = nin[l];
        if ((rc = gemm<false, false, EPI_DX>(d, st))) return rc;
        up = dp[l & 1];
    }
    return EDT_OK;
}

int sdf_mlp_adam(float* master, uint16_t* w16, float* m, float* v, const float* grad, int32_t step,
                 float lr, float beta1, float beta2, float eps, void* stream)
{
    if (!master || !w16 || !m || !v || !grad || step < 1) {
        set_error("sdf_mlp_adam: NULL pointer or step < 1");
        return EDT_ERR_ARG;
    }
    const float c1 = (float)(1.0 - std::pow((double)beta1, (double)step));
    const float c2 = (float)(1.0 - std::pow((double)beta2, (double)step));
    hipLaunchKernelGGL(k_adam, dim3((SDF_MLP_PARAMS + 255) / 256), dim3(256), 0, as_stream(stream),
                       master, w16, m, v, grad, (int)SDF_MLP_PARAMS, lr, beta1, beta2, eps, c1, c2);
    return check_launch("k_adam");
}

int sdf_mlp_fallback(const float* y, const float* radii, const float* eps_vox, int32_t batch,
                     float voxel, float margin, int32_t* need, int32_t* count, void* stream)
{
    if (!y || !radii || !eps_vox || !need || !count || batch < 1 || !(voxel > 0.0f)) {
        set_error("sdf_mlp_fallback: bad argument");
        return EDT_ERR_ARG;
    }
    const hipStream_t st = as_stream(stream);
    hipLaunchKernelGGL(k_zero_int, dim3(1), dim3(1), 0, st, count);
    int rc = check_launch("k_zero_int");
    if (rc) return rc;
    hipLaunchKernelGGL(k_fallback, dim3((batch + 255) / 256), dim3(256), 0, st, y, radii, eps_vox,
                       (int)batch, voxel, margin, need, count);
    return check_launch("k_fallback");
}

int sdf_mlp_infer(const uint16_t* w16, const float* master, const float* q, int32_t batch, float* y,
                  const float* radii, const float* eps_vox, float voxel, float margin, int32_t* need,
                  void* stream)
{
    if (!w16 || !master || !q || !y || batch < 1) {
        set_error("sdf_mlp_infer: NULL pointer or batch < 1");
        return EDT_ERR_ARG;
    }
    if (need && (!radii || !eps_vox || !(voxel > 0.0f))) {
        set_error("sdf_mlp_infer: the fallback rule needs radii, eps_vox and a voxel size > 0");
        return EDT_ERR_ARG;
    }
    hipLaunchKernelGGL(k_mlp_infer, dim3((batch + 63) / 64), dim3(512), 0, as_stream(stream), w16, master, q,
                       (int)batch, y, radii, eps_vox, voxel, margin, need);
    return check_launch("k_mlp_infer");
}

int sdf_mlp_select(const float* y, const int32_t* need, const float* exact, int32_t exact_row,
                   int32_t exact_col, int32_t batch, float* out, void* stream)
{
    if (!y || !need || !exact || !out || batch < 1 || exact_row < 0 || exact_col < 0) {
        set_error("sdf_mlp_select: NULL pointer, batch < 1 or negative stride");
        return EDT_ERR_ARG;
    }
    const int n = batch * SDF_MLP_OUT;
    hipLaunchKernelGGL(k_select, dim3((n + 255) / 256), dim3(256), 0, as_stream(stream), y, need, exact,
                       (int)exact_row, (int)exact_col, (int)batch, out);
    return check_launch("k_select");
}

int sdf_mlp_calibrate(const float* pred, const float* target, int32_t batch, float clip_vox,
                      float* eps_vox, void* stream)
{
    if (!pred || !target || !eps_vox || batch < 1) {
        set_error("sdf_mlp_calibrate: NULL pointer or batch < 1");
        return EDT_ERR_ARG;
    }
    const hipStream_t st = as_stream(stream);
    hipLaunchKernelGGL(k_zero_f32, dim3(1), dim3(64), 0, st, eps_vox, (int)SDF_MLP_OUT);
    int rc = check_launch("k_zero_f32");
    if (rc) return rc;
    const int n = batch * SDF_MLP_OUT;
    hipLaunchKernelGGL(k_calibrate, dim3((n + 255) / 256), dim3(256), 0, st, pred, target, (int)batch,
                       clip_vox, reinterpret_cast<unsigned*>(eps_vox));
    return check_launch("k_calibrate");
}

}  // extern "C"
