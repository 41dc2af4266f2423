// Host API of libedtmi.so and the small kernels of the control cycle:
// map clearing, point-cloud and link insertion (Sec. III-A) and the sphere
// query (Alg. 2 ExtractClosestObstaclePose, Eq. dist).  The distance
// transform kernels live in edt_core.hip.
#include <algorithm>
#include <climits>
#include <cmath>

#include "common.h"

namespace edtmi {

namespace {

// ---------------------------------------------------------------------------
// clear, insertion, query
// ---------------------------------------------------------------------------
// Zero n bytes: 16-byte stores over the aligned body, bytes for the
// unaligned head (< 16 bytes) and tail (< 16 bytes).
__global__ void k_fill_zero(uint8_t* p, int64_t head, int64_t body, int64_t tail)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < body) reinterpret_cast<uint4*>(p + head)[i] = make_uint4(0, 0, 0, 0);
    if (i < head) p[i] = 0;
    if (i < tail) p[head + 16 * body + i] = 0;
}

struct GridArgs {
    int nx, ny, nz;
    float ox, oy, oz, v;
};

__device__ __forceinline__ float xform_row(const float* T, int r, float px, float py, float pz)
{
    return __builtin_fmaf(T[4 * r + 2], pz,
                          __builtin_fmaf(T[4 * r + 1], py, __builtin_fmaf(T[4 * r], px, T[4 * r + 3])));
}

__device__ __forceinline__ bool discretize(float m, float o, float v, int n, int& out)
{
    const float u = (m - o) / v;
    if (!(u >= 0.0f && u < (float)n)) return false;
    out = (int)floorf(u);
    return true;
}

__device__ __forceinline__ void insert_point(const GridArgs& g, const float* T, float px, float py,
                                             float pz, uint8_t* occ, const uint8_t* exclude)
{
    const float mx = xform_row(T, 0, px, py, pz);
    const float my = xform_row(T, 1, px, py, pz);
    const float mz = xform_row(T, 2, px, py, pz);
    int ix, iy, iz;
    if (!discretize(mx, g.ox, g.v, g.nx, ix)) return;
    if (!discretize(my, g.oy, g.v, g.ny, iy)) return;
    if (!discretize(mz, g.oz, g.v, g.nz, iz)) return;
    const int64_t lin = ix + (int64_t)g.nx * (iy + (int64_t)g.ny * iz);
    if (exclude && exclude[lin]) return;
    occ[lin] = 1;
}

__global__ void k_insert_points(GridArgs g, const float* __restrict__ pts, int64_t n,
                                const float* __restrict__ T, const uint8_t* __restrict__ exclude,
                                uint8_t* __restrict__ occ)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float t[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) t[k] = T[k];
    insert_point(g, t, pts[3 * i], pts[3 * i + 1], pts[3 * i + 2], occ, exclude);
}

// Probabilistic occupancy (Sec. III-A).  One thread per point: the
// endpoint's voxel is flagged as a hit and every voxel the sensor ray
// crosses before it as free, for this frame.  The walk goes voxel by voxel
// from the sensor's voxel (Amanatides-Woo order): each step crosses the
// boundary with the smallest parameter tmax among the axes that still have
// voxels to cross, x before y before z on ties, so it ends exactly on the
// endpoint voxel.  float32, one rounding per operation, no contraction.
__global__ void k_logodds_rays(GridArgs g, const float* __restrict__ pts, int64_t n,
                               const float* __restrict__ T, const uint8_t* __restrict__ keep,
                               const uint8_t* __restrict__ exclude, uint8_t* __restrict__ hit,
                               uint8_t* __restrict__ fre)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (keep && !keep[i]) return;
    float t[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) t[k] = T[k];
    const float px = pts[3 * i], py = pts[3 * i + 1], pz = pts[3 * i + 2];
    const float o[3] = {g.ox, g.oy, g.oz};
    const int nn[3] = {g.nx, g.ny, g.nz};
    float b[3];
    int e[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const float m = xform_row(t, k, px, py, pz);
        b[k] = (m - o[k]) / g.v;
        if (!(b[k] >= 0.0f && b[k] < (float)nn[k])) return;   // also drops NaN
        e[k] = (int)floorf(b[k]);
    }
    const int64_t le = e[0] + (int64_t)g.nx * (e[1] + (int64_t)g.ny * e[2]);
    if (exclude && exclude[le]) return;
    hit[le] = 1;
    int cur[3], step[3], left[3], total = 0;
    float tmax[3], tdel[3];
    float a[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        a[k] = (t[4 * k + 3] - o[k]) / g.v;   // sensor position, voxel units
        // a sensor farther than 2^16 voxels on an axis, or not finite:
        // no crossings are walked (its hits still count)
        if (!(fabsf(a[k]) <= 65536.0f)) return;
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        cur[k] = (int)floorf(a[k]);
        const float d = b[k] - a[k];
        step[k] = e[k] > cur[k] ? 1 : (e[k] < cur[k] ? -1 : 0);
        left[k] = step[k] > 0 ? e[k] - cur[k] : cur[k] - e[k];
        total += left[k];
        if (step[k] != 0) {
            const float bound = (float)(step[k] > 0 ? cur[k] + 1 : cur[k]);
            tmax[k] = (bound - a[k]) / d;
            tdel[k] = 1.0f / fabsf(d);
        } else {
            tmax[k] = __builtin_huge_valf();
            tdel[k] = 0.0f;
        }
    }
    for (int s = 0; s < total; ++s) {
        if ((unsigned)cur[0] < (unsigned)g.nx && (unsigned)cur[1] < (unsigned)g.ny &&
            (unsigned)cur[2] < (unsigned)g.nz)
            fre[cur[0] + (int64_t)g.nx * (cur[1] + (int64_t)g.ny * cur[2])] = 1;
        int ax = left[0] > 0 ? 0 : -1;
        if (left[1] > 0 && (ax < 0 || tmax[1] < tmax[ax])) ax = 1;
        if (left[2] > 0 && (ax < 0 || tmax[2] < tmax[ax])) ax = 2;
        // one of the axes has voxels left while s < total
        cur[ax] += step[ax];
        left[ax] -= 1;
        tmax[ax] = tmax[ax] + tdel[ax];
    }
}

struct LogOdds {
    int hit, miss, lmin, lmax, threshold;
};

// One thread per 4 voxels: hit beats free, clamp, threshold, and clear the
// frame's flags for the next frame.
__global__ void k_logodds_update(int64_t n, LogOdds p, int16_t* __restrict__ L,
                                 uint8_t* __restrict__ occ, uint8_t* __restrict__ hit,
                                 uint8_t* __restrict__ fre)
{
    const int64_t i0 = 4 * ((int64_t)blockIdx.x * blockDim.x + threadIdx.x);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int64_t v = i0 + k;
        if (v >= n) return;
        int l = L[v];
        if (hit[v]) {
            l = min(l + p.hit, p.lmax);
            hit[v] = 0;
            fre[v] = 0;
        } else if (fre[v]) {
            l = max(l + p.miss, p.lmin);
            fre[v] = 0;
        }
        L[v] = (int16_t)l;
        occ[v] = l > p.threshold ? 1 : 0;
    }
}

// Static-scene reuse: flags[0] = "transform needed" for this call, flags[1]
// = "the snapshot belongs to the result in d2 / site".
__global__ void k_cache_begin(int* flags) { flags[0] = flags[1] ? 0 : 1; }
__global__ void k_cache_end(int* flags) { flags[1] = 1; }

// Compare 16 occupancy bytes per thread with the snapshot as occupied /
// free (any nonzero byte is occupied); on a difference raise the flag and
// store the new state.  ALIGNED: occ is 16-byte aligned.
template <bool ALIGNED>
__global__ void k_cache_compare(const uint8_t* __restrict__ occ, uint8_t* __restrict__ snap, int64_t n,
                                int* __restrict__ flags)
{
    const int64_t i0 = 16 * ((int64_t)blockIdx.x * blockDim.x + threadIdx.x);
    if (i0 >= n) return;
    uint8_t cur[16];
    if (ALIGNED && i0 + 16 <= n) {
        const uint4 v = *reinterpret_cast<const uint4*>(occ + i0);
        const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int k = 0; k < 16; ++k) cur[k] = (w[k >> 2] >> (8 * (k & 3))) & 0xFFu ? 1 : 0;
    } else {
#pragma unroll
        for (int k = 0; k < 16; ++k) cur[k] = (i0 + k < n && occ[i0 + k]) ? 1 : 0;
    }
    bool diff = false;
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        if (i0 + k < n && snap[i0 + k] != cur[k]) {
            snap[i0 + k] = cur[k];
            diff = true;
        }
    }
    if (diff) flags[0] = 1;
}

constexpr int MAX_LINKS = 64;
struct LinkSegs {
    int n;                       // segments (selected links)
    int link[MAX_LINKS];         // link index of segment s
    int start[MAX_LINKS];        // first point of segment s in link_pts
    int prefix[MAX_LINKS + 1];   // first thread of segment s
};

// Link point i of the selected segments, placed by its link's pose.
__device__ __forceinline__ void insert_link_point(const GridArgs& g, const float* link_pts,
                                                  const LinkSegs& segs, const float* poses, int i,
                                                  uint8_t* occ)
{
    int s = 0;
    while (s + 1 < segs.n && segs.prefix[s + 1] <= i) ++s;
    const int64_t p = segs.start[s] + (int64_t)(i - segs.prefix[s]);
    const float* T = poses + 12 * segs.link[s];
    float t[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) t[k] = T[k];
    insert_point(g, t, link_pts[3 * p], link_pts[3 * p + 1], link_pts[3 * p + 2], occ, nullptr);
}

__global__ void k_insert_links(GridArgs g, const float* __restrict__ link_pts, LinkSegs segs,
                               const float* __restrict__ poses, uint8_t* __restrict__ occ)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= segs.prefix[segs.n]) return;
    insert_link_point(g, link_pts, segs, poses, i, occ);
}

// Maps of one grid, batched over blockIdx.y: map j is occ[j] (its link poses
// at poses + j * pose_stride floats); a map whose gate is 0 is left alone.
struct MapBytes {
    uint8_t* occ[EDT_BATCH_MAX];
};

__device__ __forceinline__ bool map_gated_off(const int* gates, int j)
{
    return gates && __builtin_amdgcn_readfirstlane(gates[j]) == 0;
}

// Zero n bytes of every map: 16-byte stores over each map's aligned body,
// bytes for its head and tail.
__global__ void k_clear_many(MapBytes m, int64_t n, const int* __restrict__ gates)
{
    const int j = blockIdx.y;
    if (map_gated_off(gates, j)) return;
    uint8_t* p = m.occ[j];
    const int64_t head = min(n, (int64_t)((16 - (reinterpret_cast<uintptr_t>(p) & 15)) & 15));
    const int64_t body = (n - head) >> 4;
    const int64_t tail = n - head - 16 * body;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < body) reinterpret_cast<uint4*>(p + head)[i] = make_uint4(0, 0, 0, 0);
    if (i < head) p[i] = 0;
    if (i < tail) p[head + 16 * body + i] = 0;
}

__global__ void k_insert_links_many(GridArgs g, const float* __restrict__ link_pts, LinkSegs segs,
                                    const float* __restrict__ poses, int64_t pose_stride, MapBytes m,
                                    const int* __restrict__ gates)
{
    const int j = blockIdx.y;
    if (map_gated_off(gates, j)) return;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= segs.prefix[segs.n]) return;
    insert_link_point(g, link_pts, segs, poses + j * pose_stride, i, m.occ[j]);
}

__device__ __forceinline__ float dist_at(const int32_t* d2, int64_t lin)
{
    return sqrtf((float)d2[lin]);
}

__device__ void query_sphere(const GridArgs& g, const int32_t* __restrict__ d2,
                             const int32_t* __restrict__ site, const float* __restrict__ centres,
                             const float* __restrict__ radii, int i, edt_sphere_result_t* __restrict__ out)
{
    const float c[3] = {centres[3 * i], centres[3 * i + 1], centres[3 * i + 2]};
    const float r = radii[i];
    const float o[3] = {g.ox, g.oy, g.oz};
    const int n3[3] = {g.nx, g.ny, g.nz};
    edt_sphere_result_t res;
    res.reserved = 0.0f;
    int v[3];
    bool inside = true;
    for (int a = 0; a < 3; ++a)
        if (!discretize(c[a], o[a], g.v, n3[a], v[a])) inside = false;
    if (!inside) {
        res.d2 = 0;
        res.site = -1;
        res.vox[0] = res.vox[1] = res.vox[2] = -1;
        res.flags = EDT_Q_OUT_OF_MAP;
        res.dist_vox = 0.0f;
        res.x_c = 0.0f;
        res.clearance = -r;
        res.grad[0] = res.grad[1] = res.grad[2] = 0.0f;
        res.nearest[0] = c[0];
        res.nearest[1] = c[1];
        res.nearest[2] = c[2];
        out[i] = res;
        return;
    }
    const int64_t lin = v[0] + (int64_t)g.nx * (v[1] + (int64_t)g.ny * v[2]);
    res.d2 = d2[lin];
    res.site = site[lin];
    res.vox[0] = v[0];
    res.vox[1] = v[1];
    res.vox[2] = v[2];
    res.grad[0] = res.grad[1] = res.grad[2] = 0.0f;
    if (res.site < 0) {
        res.flags = EDT_Q_EMPTY;
        res.dist_vox = INFINITY;
        res.x_c = INFINITY;
        res.clearance = INFINITY;
        res.nearest[0] = res.nearest[1] = res.nearest[2] = INFINITY;
        out[i] = res;
        return;
    }
    res.flags = 0;
    const int s = res.site;
    const int sxyz[3] = {s % g.nx, (s / g.nx) % g.ny, s / (g.nx * g.ny)};
    float dd[3];
    for (int a = 0; a < 3; ++a) {
        res.nearest[a] = __builtin_fmaf((float)sxyz[a] + 0.5f, g.v, o[a]);
        dd[a] = res.nearest[a] - c[a];
    }
    const float xc = sqrtf(__builtin_fmaf(dd[2], dd[2], __builtin_fmaf(dd[1], dd[1], dd[0] * dd[0])));
    res.dist_vox = dist_at(d2, lin);
    res.x_c = xc;
    res.clearance = xc - r;
    const int64_t stride[3] = {1, g.nx, (int64_t)g.nx * g.ny};
    for (int a = 0; a < 3; ++a) {
        float gr;
        if (n3[a] == 1) gr = 0.0f;
        else if (v[a] == 0) gr = dist_at(d2, lin + stride[a]) - dist_at(d2, lin);
        else if (v[a] == n3[a] - 1) gr = dist_at(d2, lin) - dist_at(d2, lin - stride[a]);
        else gr = 0.5f * (dist_at(d2, lin + stride[a]) - dist_at(d2, lin - stride[a]));
        res.grad[a] = gr;
    }
    out[i] = res;
}

__global__ void k_query_spheres(GridArgs g, const int32_t* __restrict__ d2,
                                const int32_t* __restrict__ site, const float* __restrict__ centres,
                                const float* __restrict__ radii, int m,
                                edt_sphere_result_t* __restrict__ out)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    query_sphere(g, d2, site, centres, radii, i, out);
}

// The maps of a batched query or insertion, each with its own grid and
// buffers, indexed by blockIdx.y (kernel arguments: at most 3.5 KiB).
struct QueryMaps {
    GridArgs g[EDT_BATCH_MAX];
    const int32_t* d2[EDT_BATCH_MAX];
    const int32_t* site[EDT_BATCH_MAX];
    const float* centres[EDT_BATCH_MAX];
    const float* radii[EDT_BATCH_MAX];
    edt_sphere_result_t* out[EDT_BATCH_MAX];
    int m[EDT_BATCH_MAX];
};

// Sphere i of map j is thread i of row j (blockIdx.y).
__global__ void k_query_spheres_many(QueryMaps q)
{
    const int j = blockIdx.y;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= q.m[j]) return;
    query_sphere(q.g[j], q.d2[j], q.site[j], q.centres[j], q.radii[j], i, q.out[j]);
}

struct PointMaps {
    GridArgs g[EDT_BATCH_MAX];
    uint8_t* occ[EDT_BATCH_MAX];
    const float* pts[EDT_BATCH_MAX];
    const float* T[EDT_BATCH_MAX];
    int64_t n[EDT_BATCH_MAX];      // points of map j
    int64_t nvox[EDT_BATCH_MAX];   // voxels of map j
};

// Zero every map of the batch: 16-byte stores over each map's aligned body,
// bytes for its head and tail.
__global__ void k_clear_maps(PointMaps p)
{
    const int j = blockIdx.y;
    uint8_t* o = p.occ[j];
    const int64_t n = p.nvox[j];
    const int64_t head = min(n, (int64_t)((16 - (reinterpret_cast<uintptr_t>(o) & 15)) & 15));
    const int64_t body = (n - head) >> 4;
    const int64_t tail = n - head - 16 * body;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < body) reinterpret_cast<uint4*>(o + head)[i] = make_uint4(0, 0, 0, 0);
    if (i < head) o[i] = 0;
    if (i < tail) o[head + 16 * body + i] = 0;
}

// Point i of map j's cloud, placed by map j's sensor pose.
__global__ void k_insert_points_maps(PointMaps p)
{
    const int j = blockIdx.y;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= p.n[j]) return;
    const float* T = p.T[j];
    float t[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) t[k] = T[k];
    const float* q = p.pts[j];
    insert_point(p.g[j], t, q[3 * i], q[3 * i + 1], q[3 * i + 2], p.occ[j], nullptr);
}

GridArgs grid_args(const edt_grid_t* g)
{
    return GridArgs{g->nx, g->ny, g->nz, g->origin[0], g->origin[1], g->origin[2], g->voxel};
}

}  // namespace

thread_local std::string g_last_error;

void set_error(const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
}

void clear_error() { g_last_error.clear(); }

int check_grid(const edt_grid_t* g)
{
    if (!g) {
        set_error("grid is NULL");
        return EDT_ERR_ARG;
    }
    if (g->nx < 1 || g->ny < 1 || g->nz < 1 || g->nx > 1024 || g->ny > 1024 || g->nz > 1024) {
        set_error("grid dims %d x %d x %d outside 1..1024", g->nx, g->ny, g->nz);
        return EDT_ERR_SHAPE;
    }
    if ((int64_t)g->nx * g->ny * g->nz >= ((int64_t)1 << 31)) {
        set_error("grid has 2^31 or more voxels");
        return EDT_ERR_SHAPE;
    }
    if (!(g->voxel > 0.0f) || !std::isfinite(g->voxel) || !std::isfinite(g->origin[0]) ||
        !std::isfinite(g->origin[1]) || !std::isfinite(g->origin[2])) {
        set_error("voxel size must be finite and > 0, origin finite");
        return EDT_ERR_SHAPE;
    }
    return EDT_OK;
}

}  // namespace edtmi

using namespace edtmi;

extern "C" {

const char* edt_status_string(int s)
{
    switch (s) {
        case EDT_OK: return "ok";
        case EDT_ERR_ARG: return "invalid argument";
        case EDT_ERR_SHAPE: return "invalid grid shape";
        case EDT_ERR_WORKSPACE: return "workspace missing or too small";
        case EDT_ERR_HIP: return "HIP runtime error";
        case EDT_ERR_UNSUPPORTED: return "unsupported request";
        default: return "unknown status";
    }
}

const char* edt_last_error(void) { return g_last_error.c_str(); }

const char* edt_version(void) { return "edtmi 0.1 gfx950"; }

int edt_clear(const edt_grid_t* grid, uint8_t* occ, void* stream)
{
    int rc = check_grid(grid);
    if (rc) return rc;
    if (!occ) {
        set_error("edt_clear: occ is NULL");
        return EDT_ERR_ARG;
    }
    const int64_t n = grid_voxels(grid);
    const int64_t head = std::min<int64_t>(n, (16 - (int64_t)(reinterpret_cast<uintptr_t>(occ) & 15)) & 15);
    const int64_t body = (n - head) >> 4;
    const int64_t tail = n - head - 16 * body;
    const int64_t threads = std::max<int64_t>(body, 16);
    const int blocks = (int)((threads + 255) / 256);
    hipLaunchKernelGGL(k_fill_zero, dim3(blocks), dim3(256), 0, as_stream(stream), occ, head,
                       body, tail);
    return check_launch("k_fill_zero");
}

int edt_insert_points(const edt_grid_t* grid, uint8_t* occ, const float* pts, int64_t n,
                      const float* T, const uint8_t* exclude, void* stream)
{
    int rc = check_grid(grid);
    if (rc) return rc;
    if (n < 0 || (n > 0 && (!occ || !pts || !T))) {
        set_error("edt_insert_points: bad pointer or negative count");
        return EDT_ERR_ARG;
    }
    if (n == 0) return EDT_OK;
    const int64_t blocks = (n + 255) / 256;
    if (blocks > INT_MAX) {
        set_error("edt_insert_points: too many points");
        return EDT_ERR_ARG;
    }
    hipLaunchKernelGGL(k_insert_points, dim3((unsigned)blocks), dim3(256), 0, as_stream(stream),
                       grid_args(grid), pts, n, T, exclude, occ);
    return check_launch("k_insert_points");
}

size_t edt_logodds_workspace_bytes(const edt_grid_t* grid)
{
    if (check_grid(grid)) return 0;
    return (size_t)(2 * grid_voxels(grid) + 255) / 256 * 256;
}

namespace {
int fill_zero(void* p, int64_t bytes, hipStream_t st)
{
    const uintptr_t a = reinterpret_cast<uintptr_t>(p);
    int64_t head = (int64_t)((16 - (a & 15)) & 15);
    if (head > bytes) head = bytes;
    const int64_t body = (bytes - head) / 16, tail = bytes - head - 16 * body;
    const int64_t work = std::max(std::max(body, head), tail);
    if (work == 0) return EDT_OK;
    hipLaunchKernelGGL(k_fill_zero, dim3((unsigned)((work + 255) / 256)), dim3(256), 0, st,
                       static_cast<uint8_t*>(p), head, body, tail);
    return check_launch("k_fill_zero");
}
}  // namespace

int edt_logodds_reset(const edt_grid_t* grid, int16_t* logodds, void* ws, size_t ws_bytes,
                      void* stream)
{
    int rc = check_grid(grid);
    if (rc) return rc;
    if (!logodds || !ws) {
        set_error("edt_logodds_reset: NULL log-odds or workspace");
        return EDT_ERR_ARG;
    }
    if (ws_bytes < edt_logodds_workspace_bytes(grid)) {
        set_error("edt_logodds_reset: workspace of %zu bytes is below %zu", ws_bytes,
                  edt_logodds_workspace_bytes(grid));
        return EDT_ERR_WORKSPACE;
    }
    const hipStream_t st = as_stream(stream);
    rc = fill_zero(logodds, 2 * grid_voxels(grid), st);
    if (!rc) rc = fill_zero(ws, 2 * grid_voxels(grid), st);
    return rc;
}

int edt_update_logodds(const edt_grid_t* grid, int16_t* logodds, uint8_t* occ, const float* pts,
                       int64_t n, const float* T, const uint8_t* keep, const uint8_t* exclude,
                       const edt_logodds_t* params, void* ws, size_t ws_bytes, void* stream)
{
    int rc = check_grid(grid);
    if (rc) return rc;
    if (!logodds || !occ || !params || !ws || n < 0 || (n > 0 && (!pts || !T))) {
        set_error("edt_update_logodds: bad pointer or negative count");
        return EDT_ERR_ARG;
    }
    if (params->min > params->max) {
        set_error("edt_update_logodds: clamp range [%d, %d] is empty", params->min, params->max);
        return EDT_ERR_ARG;
    }
    if (ws_bytes < edt_logodds_workspace_bytes(grid)) {
        set_error("edt_update_logodds: workspace of %zu bytes is below %zu", ws_bytes,
                  edt_logodds_workspace_bytes(grid));
        return EDT_ERR_WORKSPACE;
    }
    const int64_t blocks = (n + 255) / 256;
    if (blocks > INT_MAX) {
        set_error("edt_update_logodds: too many points");
        return EDT_ERR_ARG;
    }
    const hipStream_t st = as_stream(stream);
    const int64_t nv = grid_voxels(grid);
    uint8_t* hit = static_cast<uint8_t*>(ws);
    uint8_t* fre = hit + nv;
    if (n > 0) {
        hipLaunchKernelGGL(k_logodds_rays, dim3((unsigned)blocks), dim3(256), 0, st, grid_args(grid),
                           pts, n, T, keep, exclude, hit, fre);
        if ((rc = check_launch("k_logodds_rays"))) return rc;
    }
    const LogOdds p{params->hit, params->miss, params->min, params->max, params->threshold};
    hipLaunchKernelGGL(k_logodds_update, dim3((unsigned)((nv + 1023) / 1024)), dim3(256), 0, st, nv, p,
                       logodds, occ, hit, fre);
    return check_launch("k_logodds_update");
}

}  // extern "C"

namespace {
// The selected links' point ranges (link_off, n_links, mask as for
// edt_insert_links), validated; total = their points.
int link_segments(const char* who, const int32_t* link_off, int32_t n_links, uint64_t mask,
                  const float* link_pts, LinkSegs& segs, int64_t& total)
{
    if (!link_off || n_links < 1 || n_links > MAX_LINKS) {
        set_error("%s: link_off is NULL or link count %d outside 1..%d", who, n_links, MAX_LINKS);
        return EDT_ERR_ARG;
    }
    if (link_off[0] != 0) {
        set_error("%s: link_off[0] must be 0", who);
        return EDT_ERR_ARG;
    }
    segs = LinkSegs{};
    total = 0;
    for (int l = 0; l < n_links; ++l) {
        if (link_off[l + 1] < link_off[l]) {
            set_error("%s: link_off not non-decreasing at %d", who, l);
            return EDT_ERR_ARG;
        }
        if (!((mask >> l) & 1u)) continue;
        const int cnt = link_off[l + 1] - link_off[l];
        if (cnt == 0) continue;
        segs.link[segs.n] = l;
        segs.start[segs.n] = link_off[l];
        segs.prefix[segs.n] = (int)total;
        total += cnt;
        ++segs.n;
    }
    if (total > INT_MAX - 256) {
        set_error("%s: too many link points", who);
        return EDT_ERR_ARG;
    }
    segs.prefix[segs.n] = (int)total;
    if (total > 0 && !link_pts) {
        set_error("%s: link_pts is NULL", who);
        return EDT_ERR_ARG;
    }
    return EDT_OK;
}
}  // namespace

extern "C" {

int edt_insert_links(const edt_grid_t* grid, uint8_t* occ, const float* link_pts,
                     const int32_t* link_off, int32_t n_links, const float* poses,
                     uint64_t mask, void* stream)
{
    int rc = check_grid(grid);
    if (rc) return rc;
    if (!occ || !poses) {
        set_error("edt_insert_links: occ or poses is NULL");
        return EDT_ERR_ARG;
    }
    LinkSegs segs;
    int64_t total;
    if ((rc = link_segments("edt_insert_links", link_off, n_links, mask, link_pts, segs, total))) return rc;
    if (total == 0) return EDT_OK;
    const int blocks = (int)((total + 255) / 256);
    hipLaunchKernelGGL(k_insert_links, dim3(blocks), dim3(256), 0, as_stream(stream),
                       grid_args(grid), link_pts, segs, poses, occ);
    return check_launch("k_insert_links");
}

int edt_clear_insert_links_many(const edt_grid_t* grid, uint8_t* const* occ, int32_t n_maps,
                                const float* link_pts, const int32_t* link_off, int32_t n_links,
                                const float* link_poses, uint64_t link_mask, const int32_t* gates,
                                void* stream)
{
    int rc = check_grid(grid);
    if (rc) return rc;
    if (!occ || !link_poses || n_maps < 1 || n_maps > EDT_BATCH_MAX) {
        set_error("edt_clear_insert_links_many: NULL occ or link_poses, or %d maps outside 1..%d",
                  n_maps, EDT_BATCH_MAX);
        return EDT_ERR_ARG;
    }
    LinkSegs segs;
    int64_t total;
    if ((rc = link_segments("edt_clear_insert_links_many", link_off, n_links, link_mask, link_pts, segs,
                            total)))
        return rc;
    MapBytes m;
    for (int j = 0; j < n_maps; ++j) {
        if (!occ[j]) {
            set_error("edt_clear_insert_links_many: occ[%d] is NULL", j);
            return EDT_ERR_ARG;
        }
        m.occ[j] = occ[j];
    }
    const hipStream_t st = as_stream(stream);
    const int64_t n = grid_voxels(grid);
    const int64_t threads = std::max<int64_t>(n >> 4, 16);
    hipLaunchKernelGGL(k_clear_many, dim3((unsigned)((threads + 255) / 256), n_maps), dim3(256), 0, st, m,
                       n, gates);
    if ((rc = check_launch("k_clear_many"))) return rc;
    if (total == 0) return EDT_OK;
    hipLaunchKernelGGL(k_insert_links_many, dim3((unsigned)((total + 255) / 256), n_maps), dim3(256), 0,
                       st, grid_args(grid), link_pts, segs, link_poses, (int64_t)12 * n_links, m, gates);
    return check_launch("k_insert_links_many");
}

size_t edt_workspace_bytes(const edt_grid_t* grid)
{
    (void)grid;
    return 0;
}

int edt_compute_stage(const edt_grid_t* grid, const uint8_t* occ, int32_t* d2, int32_t* site,
                      int stage, const edt_tuning_t* tuning, void* stream)
{
    int rc = check_grid(grid);
    if (rc) return rc;
    if (stage < EDT_STAGE_XY || stage > EDT_STAGE_ALL) {
        set_error("edt_compute_stage: bad stage %d", stage);
        return EDT_ERR_ARG;
    }
    if (!site || ((stage & EDT_STAGE_XY) && !occ) || ((stage & EDT_STAGE_Z) && !d2)) {
        set_error("edt_compute: NULL occ, d2 or site");
        return EDT_ERR_ARG;
    }
    const EdtTuning t = tuning ? tuning_from(tuning) : current_tuning(grid);
    if (!tile_ok(1, t.xy_tw, grid, t.xy_nt) || !tile_ok(2, t.z_tw, grid, t.z_nt)) {
        set_error("tiles (%d / %d, %d / %d) not valid for a %d x %d x %d grid", t.xy_tw, t.xy_nt,
                  t.z_tw, t.z_nt, grid->nx, grid->ny, grid->nz);
        return EDT_ERR_UNSUPPORTED;
    }
    const hipStream_t st = as_stream(stream);
    if (stage & EDT_STAGE_XY) {
        rc = launch_edt_xy(grid, occ, d2, reinterpret_cast<uint32_t*>(site), t.xy_tw, t.xy_nt, st);
        if (rc) return rc;
    }
    if (stage & EDT_STAGE_Z) rc = launch_edt_z(grid, d2, site, t.z_tw, t.z_nt, st);
    return rc;
}

int edt_compute_tuned(const edt_grid_t* grid, const uint8_t* occ, int32_t* d2, int32_t* site,
                      const edt_tuning_t* tuning, void* stream)
{
    return edt_compute_stage(grid, occ, d2, site, EDT_STAGE_ALL, tuning, stream);
}

int edt_compute(const edt_grid_t* grid, const uint8_t* occ, int32_t* d2, int32_t* site,
                void* ws, size_t ws_bytes, void* stream)
{
    (void)ws;
    (void)ws_bytes;
    return edt_compute_stage(grid, occ, d2, site, EDT_STAGE_ALL, nullptr, stream);
}

int edt_compute_many_gated(const edt_batch_map_t* maps, int32_t n_maps, const int32_t* gates,
                           const edt_tuning_t* tuning, void* stream)
{
    if (!maps || n_maps < 1 || n_maps > EDT_BATCH_MAX) {
        set_error("edt_compute_many: need 1..%d maps, got %d", EDT_BATCH_MAX, n_maps);
        return EDT_ERR_ARG;
    }
    EdtTuning t;
    if (tuning) {
        t = tuning_from(tuning);
    } else {
        edt_grid_t big = maps[0].grid;
        for (int i = 1; i < n_maps; ++i) {
            big.nx = std::max(big.nx, maps[i].grid.nx);
            big.ny = std::max(big.ny, maps[i].grid.ny);
            big.nz = std::max(big.nz, maps[i].grid.nz);
        }
        if (check_grid(&big)) return check_grid(&big);
        t = current_tuning(&big);
    }
    static thread_local EdtMapSet sxy, sz;   // ~2.7 KiB each: kept off the stack
    int rc = make_map_sets(maps, n_maps, t, sxy, sz, gates);
    if (rc) return rc;
    const hipStream_t st = as_stream(stream);
    rc = launch_edt_xy_set(sxy, t.xy_tw, t.xy_nt, st);
    if (!rc) rc = launch_edt_z_set(sz, t.z_tw, t.z_nt, st);
    return rc;
}

int edt_compute_many(const edt_batch_map_t* maps, int32_t n_maps, const edt_tuning_t* tuning,
                     void* stream)
{
    return edt_compute_many_gated(maps, n_maps, nullptr, tuning, stream);
}

size_t edt_cache_workspace_bytes(const edt_grid_t* grid)
{
    if (check_grid(grid)) return 0;
    return 256 + (size_t)(grid_voxels(grid) + 255) / 256 * 256;
}

int edt_cache_reset(const edt_grid_t* grid, void* cache, size_t cache_bytes, void* stream)
{
    int rc = check_grid(grid);
    if (rc) return rc;
    if (!cache || cache_bytes < edt_cache_workspace_bytes(grid)) {
        set_error("edt_cache_reset: cache of %zu bytes is below %zu", cache_bytes,
                  edt_cache_workspace_bytes(grid));
        return cache ? EDT_ERR_WORKSPACE : EDT_ERR_ARG;
    }
    return fill_zero(cache, (int64_t)edt_cache_workspace_bytes(grid), as_stream(stream));
}

int edt_compute_cached(const edt_grid_t* grid, const uint8_t* occ, int32_t* d2, int32_t* site,
                       void* cache, size_t cache_bytes, void* stream)
{
    int rc = check_grid(grid);
    if (rc) return rc;
    if (!occ || !d2 || !site || !cache) {
        set_error("edt_compute_cached: NULL occ, d2, site or cache");
        return EDT_ERR_ARG;
    }
    if (cache_bytes < edt_cache_workspace_bytes(grid)) {
        set_error("edt_compute_cached: cache of %zu bytes is below %zu", cache_bytes,
                  edt_cache_workspace_bytes(grid));
        return EDT_ERR_WORKSPACE;
    }
    const EdtTuning t = current_tuning(grid);
    if (!tile_ok(1, t.xy_tw, grid, t.xy_nt) || !tile_ok(2, t.z_tw, grid, t.z_nt)) {
        set_error("edt_compute_cached: no valid tiles for this grid");
        return EDT_ERR_UNSUPPORTED;
    }
    const hipStream_t st = as_stream(stream);
    int* flags = static_cast<int*>(cache);
    uint8_t* snap = static_cast<uint8_t*>(cache) + 256;
    const int64_t n = grid_voxels(grid);
    hipLaunchKernelGGL(k_cache_begin, dim3(1), dim3(1), 0, st, flags);
    if ((rc = check_launch("k_cache_begin"))) return rc;
    const unsigned blocks = (unsigned)(((n + 15) / 16 + 255) / 256);
    if ((reinterpret_cast<uintptr_t>(occ) & 15) == 0)
        hipLaunchKernelGGL(k_cache_compare<true>, dim3(blocks), dim3(256), 0, st, occ, snap, n, flags);
    else
        hipLaunchKernelGGL(k_cache_compare<false>, dim3(blocks), dim3(256), 0, st, occ, snap, n, flags);
    if ((rc = check_launch("k_cache_compare"))) return rc;
    rc = launch_edt_xy(grid, occ, d2, reinterpret_cast<uint32_t*>(site), t.xy_tw, t.xy_nt, st, flags);
    if (!rc) rc = launch_edt_z(grid, d2, site, t.z_tw, t.z_nt, st, flags);
    if (rc) return rc;
    hipLaunchKernelGGL(k_cache_end, dim3(1), dim3(1), 0, st, flags);
    return check_launch("k_cache_end");
}

int edt_query_spheres_many(const edt_batch_map_t* maps, int32_t n_maps, const float* const* centres,
                           const float* const* radii, const int32_t* m, edt_sphere_result_t* const* out,
                           void* stream)
{
    if (!maps || !centres || !radii || !m || !out || n_maps < 1 || n_maps > EDT_BATCH_MAX) {
        set_error("edt_query_spheres_many: NULL array or %d maps outside 1..%d", n_maps, EDT_BATCH_MAX);
        return EDT_ERR_ARG;
    }
    static thread_local QueryMaps q;   // 3.5 KiB: off the stack
    int m_max = 0;
    for (int j = 0; j < n_maps; ++j) {
        int rc = check_grid(&maps[j].grid);
        if (rc) return rc;
        if (m[j] < 0 || (m[j] > 0 && (!maps[j].d2 || !maps[j].site || !centres[j] || !radii[j] || !out[j]))) {
            set_error("edt_query_spheres_many: map %d: NULL buffer or negative count", j);
            return EDT_ERR_ARG;
        }
        q.g[j] = grid_args(&maps[j].grid);
        q.d2[j] = maps[j].d2;
        q.site[j] = maps[j].site;
        q.centres[j] = centres[j];
        q.radii[j] = radii[j];
        q.out[j] = out[j];
        q.m[j] = m[j];
        m_max = std::max(m_max, (int)m[j]);
    }
    if (m_max == 0) return EDT_OK;
    hipLaunchKernelGGL(k_query_spheres_many, dim3((m_max + 63) / 64, n_maps), dim3(64), 0, as_stream(stream), q);
    return check_launch("k_query_spheres_many");
}

int edt_clear_insert_points_many(const edt_grid_t* grids, uint8_t* const* occ, int32_t n_maps,
                                 const float* const* pts, const int64_t* n_pts,
                                 const float* const* T_map_sensor, void* stream)
{
    if (!grids || !occ || !pts || !n_pts || !T_map_sensor || n_maps < 1 || n_maps > EDT_BATCH_MAX) {
        set_error("edt_clear_insert_points_many: NULL array or %d maps outside 1..%d", n_maps, EDT_BATCH_MAX);
        return EDT_ERR_ARG;
    }
    static thread_local PointMaps p;   // 3.2 KiB: off the stack
    int64_t n_max = 0, v_max = 0;
    for (int j = 0; j < n_maps; ++j) {
        int rc = check_grid(&grids[j]);
        if (rc) return rc;
        if (!occ[j] || n_pts[j] < 0 || (n_pts[j] > 0 && (!pts[j] || !T_map_sensor[j]))) {
            set_error("edt_clear_insert_points_many: map %d: NULL buffer or negative count", j);
            return EDT_ERR_ARG;
        }
        if (n_pts[j] > (int64_t)INT_MAX * 256) {
            set_error("edt_clear_insert_points_many: map %d: too many points", j);
            return EDT_ERR_ARG;
        }
        p.g[j] = grid_args(&grids[j]);
        p.occ[j] = occ[j];
        p.pts[j] = pts[j];
        p.T[j] = T_map_sensor[j];
        p.n[j] = n_pts[j];
        p.nvox[j] = grid_voxels(&grids[j]);
        n_max = std::max(n_max, n_pts[j]);
        v_max = std::max(v_max, p.nvox[j]);
    }
    const hipStream_t st = as_stream(stream);
    const int64_t threads = std::max<int64_t>(v_max >> 4, 16);
    hipLaunchKernelGGL(k_clear_maps, dim3((unsigned)((threads + 255) / 256), n_maps), dim3(256), 0, st, p);
    int rc = check_launch("k_clear_maps");
    if (rc || n_max == 0) return rc;
    hipLaunchKernelGGL(k_insert_points_maps, dim3((unsigned)((n_max + 255) / 256), n_maps), dim3(256), 0, st, p);
    return check_launch("k_insert_points_maps");
}

int edt_query_spheres(const edt_grid_t* grid, const int32_t* d2, const int32_t* site,
                      const float* centres, const float* radii, int32_t m,
                      edt_sphere_result_t* out, void* stream)
{
    int rc = check_grid(grid);
    if (rc) return rc;
    if (m < 0 || (m > 0 && (!d2 || !site || !centres || !radii || !out))) {
        set_error("edt_query_spheres: bad pointer or negative count");
        return EDT_ERR_ARG;
    }
    if (m == 0) return EDT_OK;
    hipLaunchKernelGGL(k_query_spheres, dim3((m + 63) / 64), dim3(64), 0, as_stream(stream),
                       grid_args(grid), d2, site, centres, radii, m, out);
    return check_launch("k_query_spheres");
}

}  // extern "C"
