// Exact squared EDT, occupancy insertion and sphere queries for gfx950.
//
// The transform is separable (Sec. III-C, Alg. 1): the nearest site within
// each row, then along y the lower envelope of the distance functions of the
// row sites of each column (the proximate sites of step 2) queried at every
// row (step 3), then the same along z over the 2D results (step 4).  Every
// step keeps the smaller coordinate on equal distance, so with the passes in
// x, y, z order the site is the smallest linear index among equidistant
// occupied voxels.
//
// Two kernels:
//   k_edt_xy  one work-group per (z slice, tile of TW consecutive x).  Waves
//             read whole rows, turn 64 bytes into one ballot mask and find
//             each column's nearest row site with clz/ctz; the x' column tile
//             stays in LDS; the y envelope is built and queried there; the
//             2D site (x' | y' << 16) is written into the site buffer.
//   k_edt_z   one work-group per (y, tile of TW consecutive x): loads those
//             columns over all z into LDS (coalesced along x), builds each
//             column's envelope, queries every z in bands and writes d2 and
//             the final site in place.
//
// Envelope keys: a site at position p with accumulated squared distance h
// has distance function f(q) = h + (q - p)^2 = K - 2qp + q^2 with K = h + p^2.
// The site b between a and c is dominated (owns no stretch of the line) iff
// (K_c - K_b)(b - a) <= (K_b - K_a)(c - b).  A query advances to the next
// proximate site only while it is strictly closer.
#include <algorithm>
#include <climits>
#include <cmath>

#include "common.h"

namespace edtmi {

namespace {

constexpr uint32_t XY_NONE = 0xFFFFFFFFu;
constexpr uint16_t X_NONE = 0xFFFFu;
constexpr int NT = 256;  // threads per work-group of the EDT kernels

// b is dominated by its neighbours a < b < c on the envelope.
template <bool WIDE>
__device__ __forceinline__ bool dominated(int pa, int ka, int pb, int kb, int pc, int kc)
{
    if constexpr (WIDE) {
        return (int64_t)(kc - kb) * (pb - pa) <= (int64_t)(kb - ka) * (pc - pb);
    } else {
        return (kc - kb) * (pb - pa) <= (kb - ka) * (pc - pb);
    }
}

// f_next(q) < f_cur(q), with f(q) = K - 2qp (+ q^2 on both sides).
__device__ __forceinline__ bool next_closer(int p0, int k0, int p1, int k1, int q)
{
    return k1 - 2 * q * p1 < k0 - 2 * q * p0;
}

// ---------------------------------------------------------------------------
// k_edt_xy
// ---------------------------------------------------------------------------
template <int TW, bool WIDE>
__global__ __launch_bounds__(NT) void k_edt_xy(const uint8_t* __restrict__ occ,
                                               uint32_t* __restrict__ xy, int nx, int ny,
                                               int nz, int ntx)
{
    extern __shared__ uint16_t lds16[];
    uint16_t* xs = lds16;                   // [ny][TW] nearest row site x'
    uint16_t* stk = lds16 + ny * TW;        // [ny][TW] envelope positions y'
    __shared__ int s_top[TW];

    const int L = xcd_remap(blockIdx.x, nz * ntx);
    const int z = L / ntx;
    const int x0 = (L - z * ntx) * TW;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;

    // ---- step 1: nearest occupied voxel within each row (ballot + clz/ctz)
    {
        const int w0 = x0 >> 6;
        const int bit = (x0 & 63) + lane;
        const int x = x0 + lane;
        const int nwords = (nx + 63) >> 6;
        for (int y = wave; y < ny; y += NT / 64) {
            const uint8_t* row = occ + ((size_t)z * ny + y) * nx;
            uint64_t mine = 0;
            int left = -1, right = -1;
            for (int c = 0; c < nwords; ++c) {
                const int xi = c * 64 + lane;
                const bool o = xi < nx && row[xi] != 0;
                const uint64_t m = __ballot(o);
                if (c < w0) {
                    if (m) left = c * 64 + 63 - __clzll(m);
                } else if (c == w0) {
                    mine = m;
                } else if (m && right < 0) {
                    right = c * 64 + __ffsll((unsigned long long)m) - 1;
                }
            }
            if (lane < TW && x < nx) {
                const uint64_t lm = mine & ((2ull << bit) - 1ull);
                const int xl = lm ? (w0 * 64 + 63 - __clzll(lm)) : left;
                const uint64_t rm = mine & (~0ull << bit);
                const int xr = rm ? (w0 * 64 + __ffsll((unsigned long long)rm) - 1) : right;
                int best;
                if (xl < 0) best = xr;
                else if (xr < 0) best = xl;
                else best = (x - xl <= xr - x) ? xl : xr;
                xs[y * TW + lane] = best < 0 ? X_NONE : (uint16_t)best;
            }
        }
    }
    __syncthreads();

    const int col = threadIdx.x % TW;
    const int band = threadIdx.x / TW;
    constexpr int NB = NT / TW;
    const int xc = x0 + col;
    const bool live = xc < nx;

    // ---- step 2: proximate sites of each column (one thread per column)
    if (band == 0) {
        int top = 0;
        int pa = 0, ka = 0, pb = 0, kb = 0;   // cached stack[top-2], stack[top-1]
        if (live) {
            for (int yy = 0; yy < ny; ++yy) {
                const int xp = xs[yy * TW + col];
                if (xp == X_NONE) continue;
                const int dx = xc - xp;
                const int kc = dx * dx + yy * yy;
                while (top >= 2 && dominated<WIDE>(pa, ka, pb, kb, yy, kc)) {
                    --top;
                    pb = pa;
                    kb = ka;
                    if (top >= 2) {
                        pa = stk[(top - 2) * TW + col];
                        const int d = xc - xs[pa * TW + col];
                        ka = d * d + pa * pa;
                    }
                }
                stk[top * TW + col] = (uint16_t)yy;
                ++top;
                pa = pb;
                ka = kb;
                pb = yy;
                kb = kc;
            }
        }
        s_top[col] = top;
    }
    __syncthreads();

    // ---- step 3: query every row, in NB bands of rows per column
    if (!live) return;
    const int top = s_top[col];
    const int len = (ny + NB - 1) / NB;
    const int y0 = band * len;
    const int y1 = min(ny, y0 + len);
    if (y0 >= y1) return;
    uint32_t* out = xy + (size_t)z * ny * nx + xc;
    if (top == 0) {
        for (int y = y0; y < y1; ++y) out[(size_t)y * nx] = XY_NONE;
        return;
    }
    auto key = [&](int p) {
        const int d = xc - xs[p * TW + col];
        return d * d + p * p;
    };
    // first k whose successor is not strictly closer at y0 (binary search)
    int lo = 0, hi = top - 1;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        const int p0 = stk[mid * TW + col], p1 = stk[(mid + 1) * TW + col];
        if (next_closer(p0, key(p0), p1, key(p1), y0)) lo = mid + 1;
        else hi = mid;
    }
    int k = lo;
    int pk = stk[k * TW + col];
    int kk = key(pk);
    int pn = 0, kn = 0;
    if (k + 1 < top) { pn = stk[(k + 1) * TW + col]; kn = key(pn); }
    for (int y = y0; y < y1; ++y) {
        while (k + 1 < top && next_closer(pk, kk, pn, kn, y)) {
            ++k;
            pk = pn;
            kk = kn;
            if (k + 1 < top) { pn = stk[(k + 1) * TW + col]; kn = key(pn); }
        }
        out[(size_t)y * nx] = (uint32_t)xs[pk * TW + col] | ((uint32_t)pk << 16);
    }
}

// ---------------------------------------------------------------------------
// k_edt_z
// ---------------------------------------------------------------------------
template <int TW, bool WIDE>
__global__ __launch_bounds__(NT) void k_edt_z(int32_t* d2, int32_t* site, int nx, int ny,
                                              int nz, int ntx)
{
    extern __shared__ uint32_t lds32[];
    uint32_t* v = lds32;                                        // [nz][TW] packed 2D site
    uint16_t* stk = reinterpret_cast<uint16_t*>(lds32 + nz * TW);  // [nz][TW]
    __shared__ int s_top[TW];

    const int L = xcd_remap(blockIdx.x, ny * ntx);
    const int y = L / ntx;
    const int x0 = (L - y * ntx) * TW;
    const int col = threadIdx.x % TW;
    const int band = threadIdx.x / TW;
    constexpr int NB = NT / TW;
    const int xc = x0 + col;
    const bool live = xc < nx;
    const size_t plane = (size_t)nx * ny;
    const size_t base = (size_t)y * nx + xc;

    // ---- load the columns (the 2D sites written by k_edt_xy)
    const int len = (nz + NB - 1) / NB;
    const int z0 = band * len;
    const int z1 = min(nz, z0 + len);
    if (live) {
        for (int zz = z0; zz < z1; ++zz)
            v[zz * TW + col] = (uint32_t)site[base + zz * plane];
    }
    __syncthreads();

    auto key = [&](int p) {
        const uint32_t s = v[p * TW + col];
        const int dx = xc - (int)(s & 0xFFFFu);
        const int dy = y - (int)(s >> 16);
        return dx * dx + dy * dy + p * p;
    };

    // ---- step 4 (step 2 along z): proximate sites, one thread per column
    if (band == 0) {
        int top = 0;
        int pa = 0, ka = 0, pb = 0, kb = 0;
        if (live) {
            for (int zz = 0; zz < nz; ++zz) {
                if (v[zz * TW + col] == XY_NONE) continue;
                const int kc = key(zz);
                while (top >= 2 && dominated<WIDE>(pa, ka, pb, kb, zz, kc)) {
                    --top;
                    pb = pa;
                    kb = ka;
                    if (top >= 2) {
                        pa = stk[(top - 2) * TW + col];
                        ka = key(pa);
                    }
                }
                stk[top * TW + col] = (uint16_t)zz;
                ++top;
                pa = pb;
                ka = kb;
                pb = zz;
                kb = kc;
            }
        }
        s_top[col] = top;
    }
    __syncthreads();

    // ---- step 4 (step 3 along z): query every z in bands
    if (!live || z0 >= z1) return;
    const int top = s_top[col];
    if (top == 0) {
        for (int zz = z0; zz < z1; ++zz) {
            d2[base + zz * plane] = INT_MAX;
            site[base + zz * plane] = -1;
        }
        return;
    }
    int lo = 0, hi = top - 1;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        const int p0 = stk[mid * TW + col], p1 = stk[(mid + 1) * TW + col];
        if (next_closer(p0, key(p0), p1, key(p1), z0)) lo = mid + 1;
        else hi = mid;
    }
    int k = lo;
    int pk = stk[k * TW + col];
    int kk = key(pk);
    int pn = 0, kn = 0;
    if (k + 1 < top) { pn = stk[(k + 1) * TW + col]; kn = key(pn); }
    for (int zz = z0; zz < z1; ++zz) {
        while (k + 1 < top && next_closer(pk, kk, pn, kn, zz)) {
            ++k;
            pk = pn;
            kk = kn;
            if (k + 1 < top) { pn = stk[(k + 1) * TW + col]; kn = key(pn); }
        }
        const uint32_t s = v[pk * TW + col];
        d2[base + zz * plane] = kk - 2 * zz * pk + zz * zz;
        site[base + zz * plane] =
            (int32_t)((s & 0xFFFFu) + (size_t)nx * ((s >> 16) + (size_t)ny * pk));
    }
}

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

constexpr int MAX_LINKS = 64;
struct LinkSegs {
    int n;                       // segments (selected links)
    int link[MAX_LINKS];         // link index of segment s
    int start[MAX_LINKS];        // first point of segment s in link_pts
    int prefix[MAX_LINKS + 1];   // first thread of segment s
};

__global__ void k_insert_links(GridArgs g, const float* __restrict__ link_pts, LinkSegs segs,
                               const float* __restrict__ poses, uint8_t* __restrict__ occ)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= segs.prefix[segs.n]) return;
    int s = 0;
    while (s + 1 < segs.n && segs.prefix[s + 1] <= i) ++s;
    const int64_t p = segs.start[s] + (int64_t)(i - segs.prefix[s]);
    const float* T = poses + 12 * segs.link[s];
    float t[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) t[k] = T[k];
    insert_point(g, t, link_pts[3 * p], link_pts[3 * p + 1], link_pts[3 * p + 2], occ, nullptr);
}

__device__ __forceinline__ float dist_at(const int32_t* d2, int64_t lin)
{
    return sqrtf((float)d2[lin]);
}

__global__ void k_query_spheres(GridArgs g, const int32_t* __restrict__ d2,
                                const int32_t* __restrict__ site, const float* __restrict__ centres,
                                const float* __restrict__ radii, int m,
                                edt_sphere_result_t* __restrict__ out)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
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

GridArgs grid_args(const edt_grid_t* g)
{
    return GridArgs{g->nx, g->ny, g->nz, g->origin[0], g->origin[1], g->origin[2], g->voxel};
}

// Tile width so that the LDS tile stays within 64 KiB.
int xy_tile(int ny) { return ny <= 256 ? 64 : (ny <= 512 ? 32 : 16); }
int z_tile(int nz) { return nz <= 128 ? 64 : (nz <= 256 ? 32 : (nz <= 512 ? 16 : 8)); }

// Allow dynamic LDS beyond the 64 KiB default (gfx950 has 160 KiB per
// work-group).  Called once per kernel instantiation and size class; the
// margin covers the kernels' small static LDS arrays.
template <typename K>
int allow_lds(K kernel, size_t bytes, bool& done)
{
    if (done || bytes + 4096 <= 65536) return EDT_OK;
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024 - 4096);
    if (e != hipSuccess) {
        set_error("hipFuncSetAttribute(%zu bytes LDS): %s", bytes, hipGetErrorString(e));
        return EDT_ERR_HIP;
    }
    done = true;
    return EDT_OK;
}

template <int TW>
int launch_xy_t(const edt_grid_t* g, const uint8_t* occ, uint32_t* xy, bool wide, hipStream_t st)
{
    const int ntx = (g->nx + TW - 1) / TW;
    const size_t lds = (size_t)4 * TW * g->ny;
    const dim3 grid(g->nz * ntx), block(NT);
    int rc;
    if (wide) {
        static bool done = false;
        if ((rc = allow_lds(k_edt_xy<TW, true>, lds, done))) return rc;
        hipLaunchKernelGGL((k_edt_xy<TW, true>), grid, block, lds, st, occ, xy, g->nx, g->ny, g->nz, ntx);
    } else {
        static bool done = false;
        if ((rc = allow_lds(k_edt_xy<TW, false>, lds, done))) return rc;
        hipLaunchKernelGGL((k_edt_xy<TW, false>), grid, block, lds, st, occ, xy, g->nx, g->ny, g->nz, ntx);
    }
    return check_launch("k_edt_xy");
}

template <int TW>
int launch_z_t(const edt_grid_t* g, int32_t* d2, int32_t* site, bool wide, hipStream_t st)
{
    const int ntx = (g->nx + TW - 1) / TW;
    const size_t lds = (size_t)6 * TW * g->nz;
    const dim3 grid(g->ny * ntx), block(NT);
    int rc;
    if (wide) {
        static bool done = false;
        if ((rc = allow_lds(k_edt_z<TW, true>, lds, done))) return rc;
        hipLaunchKernelGGL((k_edt_z<TW, true>), grid, block, lds, st, d2, site, g->nx, g->ny, g->nz, ntx);
    } else {
        static bool done = false;
        if ((rc = allow_lds(k_edt_z<TW, false>, lds, done))) return rc;
        hipLaunchKernelGGL((k_edt_z<TW, false>), grid, block, lds, st, d2, site, g->nx, g->ny, g->nz, ntx);
    }
    return check_launch("k_edt_z");
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

// True when some cross product of the envelope test can exceed int32:
// keys reach (nx-1)^2 + (ny-1)^2 + (nz-1)^2 and positions differ by up to
// n - 1; every dimension <= 512 keeps all products below 2^31.
bool needs_wide(const edt_grid_t* g) { return g->nx > 512 || g->ny > 512 || g->nz > 512; }

int launch_edt_xy(const edt_grid_t* g, const uint8_t* occ, uint32_t* xy, hipStream_t st)
{
    const bool wide = needs_wide(g);
    switch (xy_tile(g->ny)) {
        case 64: return launch_xy_t<64>(g, occ, xy, wide, st);
        case 32: return launch_xy_t<32>(g, occ, xy, wide, st);
        default: return launch_xy_t<16>(g, occ, xy, wide, st);
    }
}

int launch_edt_z(const edt_grid_t* g, int32_t* d2, int32_t* site, hipStream_t st)
{
    const bool wide = needs_wide(g);
    switch (z_tile(g->nz)) {
        case 64: return launch_z_t<64>(g, d2, site, wide, st);
        case 32: return launch_z_t<32>(g, d2, site, wide, st);
        case 16: return launch_z_t<16>(g, d2, site, wide, st);
        default: return launch_z_t<8>(g, d2, site, wide, st);
    }
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

int edt_insert_links(const edt_grid_t* grid, uint8_t* occ, const float* link_pts,
                     const int32_t* link_off, int32_t n_links, const float* poses,
                     uint64_t mask, void* stream)
{
    int rc = check_grid(grid);
    if (rc) return rc;
    if (!occ || !link_off || !poses || n_links < 1 || n_links > MAX_LINKS) {
        set_error("edt_insert_links: bad pointer or link count %d", n_links);
        return EDT_ERR_ARG;
    }
    if (link_off[0] != 0) {
        set_error("edt_insert_links: link_off[0] must be 0");
        return EDT_ERR_ARG;
    }
    LinkSegs segs{};
    int64_t total = 0;
    for (int l = 0; l < n_links; ++l) {
        if (link_off[l + 1] < link_off[l]) {
            set_error("edt_insert_links: link_off not non-decreasing at %d", l);
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
        set_error("edt_insert_links: too many link points");
        return EDT_ERR_ARG;
    }
    segs.prefix[segs.n] = (int)total;
    if (total == 0) return EDT_OK;
    if (!link_pts) {
        set_error("edt_insert_links: link_pts is NULL");
        return EDT_ERR_ARG;
    }
    const int blocks = (int)((total + 255) / 256);
    hipLaunchKernelGGL(k_insert_links, dim3(blocks), dim3(256), 0, as_stream(stream),
                       grid_args(grid), link_pts, segs, poses, occ);
    return check_launch("k_insert_links");
}

size_t edt_workspace_bytes(const edt_grid_t* grid)
{
    (void)grid;
    return 0;
}

int edt_compute_stage(const edt_grid_t* grid, const uint8_t* occ, int32_t* d2, int32_t* site,
                      void* ws, size_t ws_bytes, int stage, void* stream)
{
    (void)ws;
    (void)ws_bytes;
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
    const hipStream_t st = as_stream(stream);
    if (stage & EDT_STAGE_XY) {
        rc = launch_edt_xy(grid, occ, reinterpret_cast<uint32_t*>(site), st);
        if (rc) return rc;
    }
    if (stage & EDT_STAGE_Z) rc = launch_edt_z(grid, d2, site, st);
    return rc;
}

int edt_compute(const edt_grid_t* grid, const uint8_t* occ, int32_t* d2, int32_t* site,
                void* ws, size_t ws_bytes, void* stream)
{
    return edt_compute_stage(grid, occ, d2, site, ws, ws_bytes, EDT_STAGE_ALL, stream);
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
