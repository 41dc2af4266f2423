// Statistical outlier filtering of a raw point cloud (Sec. III-A: the
// points are filtered by their Euclidean distance to their neighbours).
//
// Per finite point i: d_i = mean distance to its k nearest other points
// within radius R, a missing neighbour counting as R; over the finite
// points mu and the sample standard deviation sigma of d_i (exact
// fixed-point sums, so independent of the order of accumulation); keep i
// iff d_i <= mu + alpha * sigma.
//
// Neighbour search: cells slightly larger than R / 2 (1.001 R / 2), so
// every neighbour within R lies in the 5 x 5 x 5 cells around a point for
// coordinates below about 80 m.  The table is the grid of cells wrapped onto
// A x B x C buckets (powers of two, each at least 8): cells that differ by
// whole periods share a bucket, the 125 cells around any cell fall into
// distinct buckets, and the cells of an x run into consecutive ones.  Points
// are counted per bucket, the counts are scanned into bucket offsets, and the
// points are scattered into their buckets, so the points of an x run of
// cells are one contiguous range (two where the run wraps).  A query visits
// its own cell, then the 25 x runs nearest first, each trimmed to the cells
// that can still hold one of the k nearest, with one thread per point in
// bucket order.  The k smallest squared distances are kept sorted in
// registers by a compare-exchange pass per candidate.
#include <algorithm>
#include <climits>
#include <cmath>

#include "common.h"

namespace edtmi {
namespace {

constexpr int KMAX = 16;

constexpr double SCALE1 = 1099511627776.0;   // 2^40: units of d
constexpr double SCALE2 = 281474976710656.0; // 2^48: units of d^2

// Bucket of a cell: (ix mod A) + A ((iy mod B) + B (iz mod C)).
struct Wrap {
    unsigned mx, my, mz;   // A - 1, B - 1, C - 1
    int sy, sz;            // log2 A, log2 (A B)
};

struct SorLayout {
    size_t count, start, cursor, sums, spts, acc, total;
    unsigned tmask;
    Wrap wrap;
    int nsums;
};

// table size: a power of two >= 4 n, at least 1024, at most 2^23
__host__ inline SorLayout sor_layout(int64_t n)
{
    int64_t T = 1024;
    while (T < 4 * n && T < (int64_t(1) << 23)) T <<= 1;
    SorLayout L;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t at = o;
        o += (bytes + 255) / 256 * 256;
        return at;
    };
    L.count = take((size_t)T * 4);
    L.start = take((size_t)T * 4);
    L.cursor = take((size_t)T * 4);
    L.nsums = (int)(T / 1024);
    L.sums = take((size_t)L.nsums * 4);
    L.spts = take((size_t)std::max<int64_t>(n, 1) * 16);
    L.acc = take(4 * 8);
    L.total = o;
    L.tmask = (unsigned)(T - 1);
    int t = 0;
    while ((int64_t(1) << t) < T) ++t;
    // T >= 2^10, so A, B and C are each at least 8
    const int a = (t + 2) / 3, b = (t - a + 1) / 2, c = t - a - b;
    L.wrap.mx = (1u << a) - 1u;
    L.wrap.my = (1u << b) - 1u;
    L.wrap.mz = (1u << c) - 1u;
    L.wrap.sy = a;
    L.wrap.sz = a + b;
    return L;
}

__device__ __forceinline__ bool finite3(float x, float y, float z)
{
    return __builtin_isfinite(x) && __builtin_isfinite(y) && __builtin_isfinite(z);
}

__device__ __forceinline__ int cell_of(float x, float h)
{
    const float c = floorf(x / h);
    return (int)fminf(fmaxf(c, -1.0e9f), 1.0e9f);
}

__device__ __forceinline__ unsigned bucket(int ix, int iy, int iz, const Wrap& w)
{
    return ((unsigned)ix & w.mx) | (((unsigned)iy & w.my) << w.sy) | (((unsigned)iz & w.mz) << w.sz);
}

__global__ void k_sor_zero(unsigned* __restrict__ count, unsigned* __restrict__ cursor, int T,
                           unsigned long long* __restrict__ acc)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < T) {
        count[i] = 0u;
        cursor[i] = 0u;
    }
    if (i < 4) acc[i] = 0ull;
}

// Counts the finite points per bucket; a point that is not finite gets its
// mean distance (NaN) here, since the neighbour search never sees it.
__global__ void k_sor_count(const float* __restrict__ pts, int64_t n, float h, Wrap w,
                            unsigned* __restrict__ count, float* __restrict__ dmean)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float x = pts[3 * i], y = pts[3 * i + 1], z = pts[3 * i + 2];
    if (!finite3(x, y, z)) {
        dmean[i] = __builtin_nanf("");
        return;
    }
    atomicAdd(count + bucket(cell_of(x, h), cell_of(y, h), cell_of(z, h), w), 1u);
}

// exclusive scan of T counts (T a multiple of 1024): per-block scan of 1024
// values (4 per thread), one block scanning the block totals, then the add
__global__ __launch_bounds__(256) void k_scan_blocks(const unsigned* __restrict__ in,
                                                     unsigned* __restrict__ out,
                                                     unsigned* __restrict__ sums)
{
    __shared__ unsigned s[256];
    const int base = blockIdx.x * 1024 + 4 * threadIdx.x;
    const uint4 v = *reinterpret_cast<const uint4*>(in + base);
    const unsigned t = v.x + v.y + v.z + v.w;
    s[threadIdx.x] = t;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
        const unsigned add = threadIdx.x >= (unsigned)off ? s[threadIdx.x - off] : 0u;
        __syncthreads();
        s[threadIdx.x] += add;
        __syncthreads();
    }
    const unsigned ex = s[threadIdx.x] - t;
    *reinterpret_cast<uint4*>(out + base) = make_uint4(ex, ex + v.x, ex + v.x + v.y, ex + v.x + v.y + v.z);
    if (threadIdx.x == 255) sums[blockIdx.x] = s[255];
}

__global__ __launch_bounds__(1024) void k_scan_sums(unsigned* __restrict__ sums, int nb)
{
    __shared__ unsigned s[1024];
    const int per = (nb + 1023) / 1024;
    const int b0 = threadIdx.x * per;
    unsigned t = 0;
    for (int j = 0; j < per; ++j)
        if (b0 + j < nb) t += sums[b0 + j];
    s[threadIdx.x] = t;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const unsigned add = threadIdx.x >= (unsigned)off ? s[threadIdx.x - off] : 0u;
        __syncthreads();
        s[threadIdx.x] += add;
        __syncthreads();
    }
    unsigned run = s[threadIdx.x] - t;
    for (int j = 0; j < per; ++j)
        if (b0 + j < nb) {
            const unsigned c = sums[b0 + j];
            sums[b0 + j] = run;
            run += c;
        }
}

__global__ __launch_bounds__(256) void k_scan_add(unsigned* __restrict__ out,
                                                  const unsigned* __restrict__ sums)
{
    const unsigned add = sums[blockIdx.x];
    uint4* p = reinterpret_cast<uint4*>(out + blockIdx.x * 1024 + 4 * threadIdx.x);
    uint4 v = *p;
    v.x += add;
    v.y += add;
    v.z += add;
    v.w += add;
    *p = v;
}

__global__ void k_sor_scatter(const float* __restrict__ pts, int64_t n, float h, Wrap w,
                              const unsigned* __restrict__ start, unsigned* __restrict__ cursor,
                              float4* __restrict__ spts)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float x = pts[3 * i], y = pts[3 * i + 1], z = pts[3 * i + 2];
    if (!finite3(x, y, z)) return;
    const unsigned b = bucket(cell_of(x, h), cell_of(y, h), cell_of(z, h), w);
    const unsigned pos = start[b] + atomicAdd(cursor + b, 1u);
    spts[pos] = make_float4(x, y, z, __int_as_float((int)i));
}

__device__ __forceinline__ unsigned long long wave_sum(unsigned long long v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// One thread per finite point, points in bucket order (neighbouring cells
// sit side by side in spts, so a wave's points share candidate ranges).  A
// query visits its own cell, then the 25 x runs (dy, dz in -2..2) of the
// 5 x 5 x 5 cells around it, nearest first, each run a contiguous range of
// cells dx in lo..hi (its own cell left out of the own run).  That is exact:
// a point within R lies in one of the 125 cells, whose ranges are disjoint,
// so it is counted once; candidates from cells a whole period away lie
// farther than R and fail the radius test.  Once k neighbours are in hand, a
// cell whose box (widened by a rounding slack) lies farther than the current
// k-th nearest is left out: its points cannot change the k smallest
// distances, and the count m = min(found, k) is already k.  The visiting
// order changes nothing: the k smallest values are summed in ascending
// order, and the statistics are integer sums, reduced per wave before one
// atomic add per wave.
template <int K>
__global__ __launch_bounds__(256) void k_sor_knn(int k, float R, float h, Wrap w, unsigned T,
                                                 const unsigned* __restrict__ start,
                                                 const unsigned* __restrict__ count,
                                                 const float4* __restrict__ spts,
                                                 float* __restrict__ dmean,
                                                 unsigned long long* __restrict__ acc)
{
    const unsigned t = blockIdx.x * blockDim.x + threadIdx.x;
    const unsigned nfin = start[T - 1] + count[T - 1];
    unsigned long long a1 = 0, a2 = 0, a3 = 0;
    if (t < nfin) {
        const float4 P = spts[t];
        const int i = __float_as_int(P.w);
        const float px = P.x, py = P.y, pz = P.z;
        const float rr = R * R;
        const int cx = cell_of(px, h), cy = cell_of(py, h), cz = cell_of(pz, h);
        // a point's cell can differ from its coordinates' box by rounding;
        // the pruning bound below is shrunk by this slack
        const float slack = 1e-4f * h + 1e-6f * (fabsf(px) + fabsf(py) + fabsf(pz));
        float best[K];
#pragma unroll
        for (int u = 0; u < K; ++u) best[u] = __builtin_huge_valf();
        int found = 0;
        auto scan = [&](unsigned e0, unsigned e1) {
            // candidates eight at a time: the eight loads are in flight together
            for (unsigned e = e0; e < e1; e += 8) {
                float4 q[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) q[u] = spts[min(e + u, e1 - 1)];
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    if (e + u >= e1 || __float_as_int(q[u].w) == i) continue;
                    const float ex = q[u].x - px, ey = q[u].y - py, ez = q[u].z - pz;
                    float sd = (ex * ex + ey * ey) + ez * ez;
                    if (!(sd <= rr)) continue;
                    ++found;
                    // no smaller than the largest kept value: best[] would not change
                    if (sd >= best[K - 1]) continue;
                    // one compare-exchange pass keeps best[] sorted ascending
#pragma unroll
                    for (int u2 = 0; u2 < K; ++u2) {
                        const float lo = fminf(best[u2], sd), hi = fmaxf(best[u2], sd);
                        best[u2] = lo;
                        sd = hi;
                    }
                }
            }
        };
        // the cells x0..x1 (offsets from cx, x0 <= x1) of one row: one range,
        // or two where the run wraps round the table
        auto scan_cells = [&](unsigned row, int x0, int x1) {
            const unsigned xs = (unsigned)(cx + x0) & w.mx, xe = (unsigned)(cx + x1) & w.mx;
            const bool wraps = xs > xe;
            const unsigned ea = wraps ? w.mx : xe;
            unsigned r0 = start[row | xs], r1 = start[row | ea] + count[row | ea];
            unsigned s0 = wraps ? start[row] : 0u, s1 = wraps ? start[row | xe] + count[row | xe] : 0u;
#pragma unroll 1
            for (int part = 0; part < 2; ++part) {
                scan(r0, r1);
                r0 = s0;
                r1 = s1;
            }
        };
        // distance from the point to the box of the cell at offset o along one
        // axis (0 for its own cell), less the slack
        auto gap = [&](int o, int cc, float pp) {
            const float lo = (float)(cc + o) * h, hi = (float)(cc + o + 1) * h;
            const float gg = o < 0 ? pp - hi : (o > 0 ? lo - pp : 0.0f);
            return fmaxf(gg - slack, 0.0f);
        };
        auto kth = [&]() {
            float v = __builtin_huge_valf();
#pragma unroll
            for (int u = 0; u < K; ++u)
                if (u == k - 1) v = best[u];
            return found >= k ? v : __builtin_huge_valf();
        };
        // the own cell
        scan_cells(bucket(0, cy, cz, w), 0, 0);
        // the 25 runs, nearest first: (dy, dz) by |dy| + |dz|, then max
        constexpr int RY[25] = {0, -1, 1, 0, 0, -1, 1, -1, 1, -2, 2, 0, 0, -2, 2, -2, 2, -1, 1, -1, 1, -2, 2, -2, 2};
        constexpr int RZ[25] = {0, 0, 0, -1, 1, -1, -1, 1, 1, 0, 0, -2, 2, -1, -1, 1, 1, -2, -2, 2, 2, -2, -2, 2, 2};
#pragma unroll 1
        for (int r = 0; r < 25; ++r) {
            const int oy = RY[r], oz = RZ[r];
            const float gy = gap(oy, cy, py), gz = gap(oz, cz, pz);
            const float base = gy * gy + gz * gz;
            const float kb = kth();
            if (base > kb) continue;
            // the x offsets still within reach: gaps grow with |dx|
            int x0 = -2, x1 = 2;
            while (x0 < 0) {
                const float g = gap(x0, cx, px);
                if (base + g * g <= kb) break;
                ++x0;
            }
            while (x1 > 0) {
                const float g = gap(x1, cx, px);
                if (base + g * g <= kb) break;
                --x1;
            }
            const unsigned row = bucket(0, cy + oy, cz + oz, w);
            if (r == 0) {   // the own run without the own cell
                if (x0 < 0) scan_cells(row, x0, -1);
                if (x1 > 0) scan_cells(row, 1, x1);
            } else {
                scan_cells(row, x0, x1);
            }
        }
        const int m = min(found, k);
        float sum = 0.0f;
#pragma unroll
        for (int u = 0; u < K; ++u)
            if (u < m) sum = sum + sqrtf(best[u]);
        sum = sum + (float)(k - m) * R;
        const float d = sum / (float)k;
        dmean[i] = d;
        const double dd = (double)d;
        a1 = (unsigned long long)(long long)rint(dd * SCALE1);
        a2 = (unsigned long long)(long long)rint(dd * dd * SCALE2);
        a3 = 1ull;
    }
    a1 = wave_sum(a1);
    a2 = wave_sum(a2);
    a3 = wave_sum(a3);
    if ((threadIdx.x & 63) == 0 && a3) {
        atomicAdd(acc + 0, a1);
        atomicAdd(acc + 1, a2);
        atomicAdd(acc + 2, a3);
    }
}

__device__ __forceinline__ double sor_threshold(const unsigned long long* acc, double alpha,
                                                double* mu_out, double* sigma_out)
{
    const long long S1 = (long long)acc[0], S2 = (long long)acc[1], cnt = (long long)acc[2];
    double mu = 0.0, sigma = 0.0;
    if (cnt > 0) mu = (double)S1 / SCALE1 / (double)cnt;
    if (cnt > 1) {
        const double var = ((double)S2 / SCALE2 - (double)cnt * mu * mu) / (double)(cnt - 1);
        sigma = var > 0.0 ? sqrt(var) : 0.0;
    }
    *mu_out = mu;
    *sigma_out = sigma;
    return mu + alpha * sigma;
}

__global__ void k_sor_keep(const float* __restrict__ pts, int64_t n, const float* __restrict__ dmean,
                           const unsigned long long* __restrict__ acc, double alpha,
                           uint8_t* __restrict__ keep, double* __restrict__ stats)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double mu, sigma;
    const double thr = sor_threshold(acc, alpha, &mu, &sigma);
    if (i == 0 && stats) {
        stats[0] = mu;
        stats[1] = sigma;
        stats[2] = thr;
    }
    if (i >= n) return;
    const bool fin = finite3(pts[3 * i], pts[3 * i + 1], pts[3 * i + 2]);
    keep[i] = fin && (double)dmean[i] <= thr ? 1 : 0;
}

}  // namespace
}  // namespace edtmi

using namespace edtmi;

extern "C" {

size_t edt_outlier_workspace_bytes(int64_t n_points)
{
    if (n_points < 0 || n_points > EDT_OUTLIER_MAX_POINTS) return 0;
    return sor_layout(n_points).total + (size_t)std::max<int64_t>(n_points, 1) * 4;
}

constexpr double OUTLIER_SUM2_MAX = 32000.0;     // m^2, below 2^15
constexpr double OUTLIER_SUM1_MAX = 8000000.0;   // m, below 2^23

int edt_outlier_filter(const float* pts, int64_t n, int32_t k, float radius, float alpha,
                       uint8_t* keep, float* mean_dist, double* stats, void* ws, size_t ws_bytes,
                       void* stream)
{
    if (n < 0 || n > EDT_OUTLIER_MAX_POINTS || (n > 0 && (!pts || !keep)) || !ws) {
        set_error("edt_outlier_filter: bad pointer or point count (0..%d)", EDT_OUTLIER_MAX_POINTS);
        return EDT_ERR_ARG;
    }
    if (k < 1 || k > KMAX || !(radius > 0.0f) || !std::isfinite(radius) || !std::isfinite(alpha)) {
        set_error("edt_outlier_filter: need 1 <= k <= %d, a finite radius > 0 and a finite alpha", KMAX);
        return EDT_ERR_ARG;
    }
    // every d_i is at most the radius, so the fixed-point sums (d_i in units
    // of 2^-40, d_i^2 in units of 2^-48) stay below 2^63 while n * radius^2
    // and n * radius stay below 2^15 m^2 and 2^23 m; a margin keeps rounding
    // of the last unit inside
    if ((double)n * (double)radius * (double)radius >= OUTLIER_SUM2_MAX ||
        (double)n * (double)radius >= OUTLIER_SUM1_MAX) {
        set_error("edt_outlier_filter: n * radius^2 = %g m^2 reaches %g (the exact sums would overflow)",
                  (double)n * (double)radius * (double)radius, OUTLIER_SUM2_MAX);
        return EDT_ERR_ARG;
    }
    if (ws_bytes < edt_outlier_workspace_bytes(n)) {
        set_error("edt_outlier_filter: workspace of %zu bytes is below %zu", ws_bytes,
                  edt_outlier_workspace_bytes(n));
        return EDT_ERR_WORKSPACE;
    }
    const SorLayout L = sor_layout(n);
    char* w = static_cast<char*>(ws);
    unsigned* count = reinterpret_cast<unsigned*>(w + L.count);
    unsigned* start = reinterpret_cast<unsigned*>(w + L.start);
    unsigned* cursor = reinterpret_cast<unsigned*>(w + L.cursor);
    unsigned* sums = reinterpret_cast<unsigned*>(w + L.sums);
    float4* spts = reinterpret_cast<float4*>(w + L.spts);
    unsigned long long* acc = reinterpret_cast<unsigned long long*>(w + L.acc);
    float* dm = mean_dist ? mean_dist : reinterpret_cast<float*>(w + L.total);
    const int T = (int)L.tmask + 1;
    const float h = radius * 0.5005f;
    const hipStream_t st = as_stream(stream);
    const unsigned pblocks = (unsigned)((std::max<int64_t>(n, 1) + 255) / 256);
    hipLaunchKernelGGL(k_sor_zero, dim3((T + 255) / 256), dim3(256), 0, st, count, cursor, T, acc);
    int rc = check_launch("k_sor_zero");
    if (rc) return rc;
    if (n > 0) {
        hipLaunchKernelGGL(k_sor_count, dim3(pblocks), dim3(256), 0, st, pts, n, h, L.wrap, count, dm);
        if ((rc = check_launch("k_sor_count"))) return rc;
    }
    hipLaunchKernelGGL(k_scan_blocks, dim3(L.nsums), dim3(256), 0, st, count, start, sums);
    if ((rc = check_launch("k_scan_blocks"))) return rc;
    hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(1024), 0, st, sums, L.nsums);
    if ((rc = check_launch("k_scan_sums"))) return rc;
    hipLaunchKernelGGL(k_scan_add, dim3(L.nsums), dim3(256), 0, st, start, sums);
    if ((rc = check_launch("k_scan_add"))) return rc;
    if (n > 0) {
        hipLaunchKernelGGL(k_sor_scatter, dim3(pblocks), dim3(256), 0, st, pts, n, h, L.wrap, start,
                           cursor, spts);
        if ((rc = check_launch("k_sor_scatter"))) return rc;
        if (k <= 8)
            hipLaunchKernelGGL(k_sor_knn<8>, dim3(pblocks), dim3(256), 0, st, (int)k, radius, h, L.wrap,
                               (unsigned)T, start, count, spts, dm, acc);
        else
            hipLaunchKernelGGL(k_sor_knn<KMAX>, dim3(pblocks), dim3(256), 0, st, (int)k, radius, h, L.wrap,
                               (unsigned)T, start, count, spts, dm, acc);
        if ((rc = check_launch("k_sor_knn"))) return rc;
    }
    hipLaunchKernelGGL(k_sor_keep, dim3(pblocks), dim3(256), 0, st, pts, n, dm, acc, (double)alpha,
                       keep, stats);
    return check_launch("k_sor_keep");
}

}  // extern "C"
