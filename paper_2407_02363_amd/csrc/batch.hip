// Many maps of uneven size in one persistent launch.
//
// The work of a batch is a queue of tiles: every xy tile of every map, then
// every z tile of every map.  Work-groups stay resident and take the next
// tile from a global counter until the queue is empty.  A map's z tiles need
// all of its xy tiles: each finished xy tile raises the map's counter with a
// release (device scope), and a work-group that takes a z tile waits until
// the counter is complete with an acquire.  Every xy tile is dequeued before
// any z tile and is being processed by a resident work-group, so the waits
// always end; they are still bounded by a spin limit, past which the tile is
// skipped and an error flag is raised in the workspace (edt_batch_status).
//
// Batches whose maps all fit the lean tiles (every axis <= 512, rows of 64
// voxels or more, up to 256 rows and 128 slices) go through a second
// persistent kernel with three phases: the row records of every map, then
// the lean xy tiles of every map (a map's wait for its records), then the
// lean z tiles of every map, two per work-group (a map's wait for its xy
// tiles).
//
// Workspace (unsigned words): [0] queue head, [1] error flag,
// [2 + m] finished record items (lean) or xy tiles (general) of map m,
// [2 + n + m] finished xy tiles of map m (lean).  A small fill kernel zeroes
// it before every launch, so the pair of launches can be captured into a
// graph.
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "edt_lean.h"

namespace edtmi {

namespace {

using namespace tiles;

struct MapDesc {
    int nx, ny, nz;
    int ntx_xy, ntx_z;       // column tiles per slice / per row
    int xy_begin, xy_count;  // queue range of the map's xy tiles
    int z_begin;             // queue start of its z tiles
    const uint8_t* occ;
    int32_t* d2;
    int32_t* site;
};

struct BatchArgs {
    int n_maps;
    int n_xy;       // xy tiles of all maps (they come first in the queue)
    int n_total;    // all tiles
    MapDesc m[EDT_BATCH_MAX];
};

constexpr int WS_HEAD = 0, WS_ERR = 1, WS_DONE = 2;

__global__ void k_batch_reset(unsigned* ws, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) ws[i] = 0u;
}

// The batch's flag of a wait that gave up, copied into a caller's int.
__global__ void k_batch_flag_out(const unsigned* ws, int32_t* out)
{
    if (threadIdx.x == 0) *out = ws[WS_ERR] ? 1 : 0;
}

// At most 128 VGPRs, so that 4 waves fit per SIMD: the LDS of the larger
// tiles allows 4 work-groups per CU, and the register allocator would
// otherwise take more for the fused xy + z body than either part needs.
template <int TXY, int TZ>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(4)))
void k_edt_batched(BatchArgs a, unsigned* ws, unsigned spin_limit)
{
    extern __shared__ uint32_t lds[];
    __shared__ int s_item;
    __shared__ int s_ok;
    for (;;) {
        __syncthreads();   // the previous tile's LDS reads are done
        if (threadIdx.x == 0) s_item = (int)atomicAdd(&ws[WS_HEAD], 1u);
        __syncthreads();
        const int it = __builtin_amdgcn_readfirstlane(s_item);
        if (it >= a.n_total) break;
        if (it < a.n_xy) {
            int m = 0;
            while (m + 1 < a.n_maps && a.m[m + 1].xy_begin <= it) ++m;
            const MapDesc& d = a.m[m];
            uint32_t* xy = reinterpret_cast<uint32_t*>(d.site);
            edt_xy_tile<TXY, false>(d.occ, xy, d.nx, d.ny, d.nz, d.ntx_xy, it - d.xy_begin, lds);
            __syncthreads();   // every thread's stores of this tile are issued
            if (threadIdx.x == 0) {
                __threadfence();
                atomicAdd(&ws[WS_DONE + m], 1u);
            }
        } else {
            int m = 0;
            while (m + 1 < a.n_maps && a.m[m + 1].z_begin <= it) ++m;
            const MapDesc& d = a.m[m];
            if (threadIdx.x == 0) {
                int ok = 1;
                unsigned spins = 0;
                while (__hip_atomic_load(&ws[WS_DONE + m], __ATOMIC_ACQUIRE,
                                         __HIP_MEMORY_SCOPE_AGENT) < (unsigned)d.xy_count) {
                    __builtin_amdgcn_s_sleep(8);
                    if (++spins > spin_limit) {
                        ok = 0;
                        atomicOr(&ws[WS_ERR], 1u);
                        break;
                    }
                }
                s_ok = ok;
            }
            __syncthreads();
            if (s_ok) edt_z_tile<TZ, false>(d.d2, d.site, d.nx, d.ny, d.nz, d.ntx_z, it - d.z_begin, lds);
        }
    }
}

// ---- lean batches
struct LeanMap {
    const uint8_t* occ;
    int32_t* d2;
    int32_t* site;
    int nx, ny, nz;
    int ntx;                 // 64-column tiles per row
    int per;                 // record rows per wave
    int waves;               // record waves of the map
    int r_begin, r_count;    // queue range of its record items (8 waves each)
    int x_begin, x_count;    // its xy tiles
    int z_begin, z_count;    // its z items (two z tiles each)
};

struct LeanArgs {
    int n_maps;
    int n_r;       // record items of all maps (first in the queue)
    int n_rx;      // record and xy items
    int n_total;   // all items
    int r_chunk;   // record items per dequeue
    int t_chunk;   // xy or z items per dequeue
    LeanMap m[EDT_BATCH_MAX];
};

// Thread 0 waits until counter reaches target (acquire, device scope),
// bounded by spin_limit; every thread learns whether it did.
__device__ __forceinline__ bool wait_count(unsigned* ws, int counter, unsigned target, unsigned spin_limit,
                                           int* s_ok)
{
    if (threadIdx.x == 0) {
        int ok = 1;
        unsigned spins = 0;
        while (__hip_atomic_load(&ws[counter], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < target) {
            __builtin_amdgcn_s_sleep(8);
            if (++spins > spin_limit) {
                ok = 0;
                atomicOr(&ws[WS_ERR], 1u);
                break;
            }
        }
        *s_ok = ok;
    }
    __syncthreads();
    return *s_ok != 0;
}

// Raises counter once every thread's stores of the item are issued (release).
__device__ __forceinline__ void release_count(unsigned* ws, int counter)
{
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        atomicAdd(&ws[counter], 1u);
    }
}

// A work-group takes a chunk of consecutive items per dequeue: r_chunk
// record items while the queue head h is below the number of record chunks
// n_rc, then t_chunk tile items from item n_r + (h - n_rc) t_chunk.  The host
// sizes the chunks so that every work-group still gets several of them:
// chunks share one atomic and one barrier among their items on large
// batches, and a small batch keeps one item per dequeue so that its items
// spread over every work-group.
__global__ __launch_bounds__(512) void k_edt_batched_lean(LeanArgs a, unsigned* ws, unsigned spin_limit)
{
    __shared__ union {
        lean::XyLds xy;
        lean::ZLds z[2];
    } u;
    __shared__ int s_item;
    __shared__ int s_ok;
    const int n = a.n_maps;
    const int n_rc = (a.n_r + a.r_chunk - 1) / a.r_chunk;
    int it = 0, left = 0;
    for (;;) {
        __syncthreads();   // the previous item's LDS use is over
        if (left == 0) {
            if (threadIdx.x == 0) s_item = (int)atomicAdd(&ws[WS_HEAD], 1u);
            __syncthreads();
            const int h = __builtin_amdgcn_readfirstlane(s_item);
            if (h < n_rc) {
                it = h * a.r_chunk;
                left = min(a.r_chunk, a.n_r - it);
            } else {
                it = a.n_r + (h - n_rc) * a.t_chunk;
                left = max(1, min(a.t_chunk, a.n_total - it));
            }
        } else {
            ++it;
        }
        --left;
        if (it >= a.n_total) break;
        if (it < a.n_r) {
            // 8 record waves: wave w of the work-group takes record wave 8 (it - r_begin) + w
            int m = 0;
            while (m + 1 < n && a.m[m + 1].r_begin <= it) ++m;
            const LeanMap& d = a.m[m];
            const int wv = __builtin_amdgcn_readfirstlane((it - d.r_begin) * 8 + (int)(threadIdx.x >> 6));
            if (wv < d.waves) {
                const int row0 = wv * d.per;
                const int nrows = min(d.per, d.ny * d.nz - row0);
                if (record_words(d.occ, d.nx))
                    row_summary_words(d.occ, d.nx, (size_t)row0, nrows, row_records(d.d2, d.nx, d.ny, d.nz));
                else
                    row_summary(d.occ, d.nx, (size_t)row0, nrows, row_records(d.d2, d.nx, d.ny, d.nz));
            }
            release_count(ws, WS_DONE + m);
        } else if (it < a.n_rx) {
            int m = 0;
            while (m + 1 < n && a.m[m + 1].x_begin <= it) ++m;
            const LeanMap& d = a.m[m];
            if (wait_count(ws, WS_DONE + m, (unsigned)d.r_count, spin_limit, &s_ok))
                lean::xy_tile(row_records(d.d2, d.nx, d.ny, d.nz), reinterpret_cast<uint32_t*>(d.site), d.nx, d.ny,
                              d.ntx, it - d.x_begin, u.xy);
            release_count(ws, WS_DONE + n + m);
        } else {
            // two z tiles of one map, one per half of the work-group; a half
            // without a tile only takes part in the barriers
            int m = 0;
            while (m + 1 < n && a.m[m + 1].z_begin <= it) ++m;
            const LeanMap& d = a.m[m];
            const bool ok = wait_count(ws, WS_DONE + n + m, (unsigned)d.x_count, spin_limit, &s_ok);
            const int h = (int)(threadIdx.x >> 8);
            const int tile = (it - d.z_begin) * 2 + h;
            const bool act = ok && tile < d.ny * d.ntx;
            lean::z_tile(d.d2, d.site, d.nx, d.ny, act ? d.nz : 0, d.ntx, act ? tile : 0, (int)(threadIdx.x & 255),
                         u.z[h]);
        }
    }
}

// Every map fits the lean tiles (and has its d2 for the records).
bool lean_batch_ok(const edt_batch_map_t* maps, int n)
{
    for (int i = 0; i < n; ++i) {
        const edt_grid_t& g = maps[i].grid;
        if (g.nx < 64 || g.nx > 512 || g.ny > lean::XY_MAX || g.nz > lean::Z_MAX || !maps[i].d2) return false;
    }
    return true;
}

int make_lean_plan(const edt_batch_map_t* maps, int n, LeanArgs& a)
{
    a.n_maps = n;
    int q = 0;
    for (int i = 0; i < n; ++i) {
        const edt_grid_t& g = maps[i].grid;
        LeanMap& d = a.m[i];
        d.occ = maps[i].occ;
        d.d2 = maps[i].d2;
        d.site = maps[i].site;
        d.nx = g.nx;
        d.ny = g.ny;
        d.nz = g.nz;
        d.ntx = (g.nx + 63) / 64;
        d.per = record_rows_per_wave(d.occ, d.nx);
        d.waves = (g.ny * g.nz + d.per - 1) / d.per;
        d.r_begin = q;
        d.r_count = (d.waves + 7) / 8;
        q += d.r_count;
    }
    a.n_r = q;
    for (int i = 0; i < n; ++i) {
        LeanMap& d = a.m[i];
        d.x_begin = q;
        d.x_count = d.nz * d.ntx;
        q += d.x_count;
    }
    a.n_rx = q;
    for (int i = 0; i < n; ++i) {
        LeanMap& d = a.m[i];
        d.z_begin = q;
        d.z_count = (d.ny * d.ntx + 1) / 2;
        q += d.z_count;
    }
    a.n_total = q;
    a.r_chunk = a.t_chunk = 1;   // sized for the grid at launch
    return EDT_OK;
}

struct BatchPlan {
    BatchArgs args;
    int nx_max, ny_max, nz_max;
    bool lean;
    LeanArgs largs;
};

int make_plan(const edt_batch_map_t* maps, int n, int txy, int tz, BatchPlan& p)
{
    p.args.n_maps = n;
    p.nx_max = p.ny_max = p.nz_max = 0;
    int q = 0;
    for (int i = 0; i < n; ++i) {
        const edt_grid_t* g = &maps[i].grid;
        int rc = check_grid(g);
        if (rc) return rc;
        if (g->nx > 512 || g->ny > 512 || g->nz > 512) {
            set_error("edt_compute_batched: map %d has an axis above 512 voxels", i);
            return EDT_ERR_UNSUPPORTED;
        }
        if (!maps[i].occ || !maps[i].d2 || !maps[i].site) {
            set_error("edt_compute_batched: NULL buffer in map %d", i);
            return EDT_ERR_ARG;
        }
        MapDesc& d = p.args.m[i];
        d.nx = g->nx;
        d.ny = g->ny;
        d.nz = g->nz;
        d.ntx_xy = (g->nx + txy - 1) / txy;
        d.ntx_z = (g->nx + tz - 1) / tz;
        d.xy_begin = q;
        d.xy_count = g->nz * d.ntx_xy;
        q += d.xy_count;
        d.occ = maps[i].occ;
        d.d2 = maps[i].d2;
        d.site = maps[i].site;
        p.nx_max = std::max(p.nx_max, g->nx);
        p.ny_max = std::max(p.ny_max, g->ny);
        p.nz_max = std::max(p.nz_max, g->nz);
    }
    p.args.n_xy = q;
    for (int i = 0; i < n; ++i) {
        MapDesc& d = p.args.m[i];
        d.z_begin = q;
        q += d.ny * d.ntx_z;
    }
    p.args.n_total = q;
    return EDT_OK;
}

EdtTuning batch_default(int nx, int ny, int nz)
{
    edt_grid_t g{nx, ny, nz, {0.0f, 0.0f, 0.0f}, 1.0f};
    EdtTuning t = default_tuning(&g);
    if (t.xy_tw > 32) t.xy_tw = 32;
    if (t.z_tw < 16) t.z_tw = 16;
    return t;
}

EdtTuning batch_current(int n, int nx, int ny, int nz, bool lean_ok)
{
    EdtTuning t;
    if (tuned_lookup(1, n, nx, ny, nz, t) && (t.xy_tw != 64 || lean_ok)) return t;
    return lean_ok ? EdtTuning{64, 64, 512, 512} : batch_default(nx, ny, nz);
}

template <int TXY, int TZ>
int launch_batched_tz(const BatchPlan& p, unsigned* ws, hipStream_t st)
{
    auto kern = k_edt_batched<TXY, TZ>;
    const size_t lds = std::max(xy_lds(TXY, p.ny_max), z_lds(TZ, p.nz_max));
    static bool lds_ok = false;
    static int per_cu = 0;
    static int n_cu = 0;
    if (!lds_ok) {
        if (hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024 - 8192) != hipSuccess) {
            set_error("edt_compute_batched: hipFuncSetAttribute failed");
            return EDT_ERR_HIP;
        }
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
            set_error("edt_compute_batched: device query failed");
            return EDT_ERR_HIP;
        }
        lds_ok = true;
    }
    // resident work-groups for this LDS size (recomputed: it depends on the batch)
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(kern), NT,
                                                     lds) != hipSuccess || per_cu < 1)
        per_cu = 1;
    const int grid = std::max(1, std::min(p.args.n_total, per_cu * n_cu));
    const int nws = WS_DONE + p.args.n_maps;
    hipLaunchKernelGGL(k_batch_reset, dim3((nws + 63) / 64), dim3(64), 0, st, ws, nws);
    int rc = check_launch("k_batch_reset");
    if (rc) return rc;
    // about 0.5 s of 8-slot sleeps before a wait gives up
    const unsigned spin_limit = 1u << 21;
    hipLaunchKernelGGL(kern, dim3(grid), dim3(NT), lds, st, p.args, ws, spin_limit);
    return check_launch("k_edt_batched");
}

int launch_batched_lean(const BatchPlan& p, unsigned* ws, hipStream_t st)
{
    static int per_cu = 0;
    static int n_cu = 0;
    if (!n_cu) {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(k_edt_batched_lean),
                                                         512, 0) != hipSuccess) {
            n_cu = 0;
            set_error("edt_compute_batched: device query failed");
            return EDT_ERR_HIP;
        }
        if (per_cu < 1) per_cu = 1;
    }
    const int slots = per_cu * n_cu;
    const int grid = std::max(1, std::min(p.largs.n_total, slots));
    // chunks of up to 4 items once every work-group gets at least 2 record
    // chunks and 8 tile chunks (measured on 32 uneven maps against 2 maps)
    LeanArgs la = p.largs;
    la.r_chunk = std::max(1, std::min(4, la.n_r / (2 * slots)));
    la.t_chunk = std::max(1, std::min(4, (la.n_total - la.n_r) / (8 * slots)));
    const int nws = WS_DONE + 2 * la.n_maps;
    hipLaunchKernelGGL(k_batch_reset, dim3((nws + 63) / 64), dim3(64), 0, st, ws, nws);
    int rc = check_launch("k_batch_reset");
    if (rc) return rc;
    const unsigned spin_limit = 1u << 21;   // about 0.5 s of 8-slot sleeps
    hipLaunchKernelGGL(k_edt_batched_lean, dim3(grid), dim3(512), 0, st, la, ws, spin_limit);
    return check_launch("k_edt_batched_lean");
}

// The lean batch kernel stands for the tile pair (64, 64).
constexpr int LEAN_TILE = 64;

int launch_batched(const BatchPlan& p, int txy, int tz, unsigned* ws, hipStream_t st)
{
    if (txy == LEAN_TILE && tz == LEAN_TILE && p.lean) return launch_batched_lean(p, ws, st);
    if (txy == 32) {
        if (tz == 64) return launch_batched_tz<32, 64>(p, ws, st);
        if (tz == 32) return launch_batched_tz<32, 32>(p, ws, st);
        if (tz == 16) return launch_batched_tz<32, 16>(p, ws, st);
    } else if (txy == 16) {
        if (tz == 64) return launch_batched_tz<16, 64>(p, ws, st);
        if (tz == 32) return launch_batched_tz<16, 32>(p, ws, st);
        if (tz == 16) return launch_batched_tz<16, 16>(p, ws, st);
    }
    set_error("edt_compute_batched: tiles (%d, %d) not available for batches", txy, tz);
    return EDT_ERR_UNSUPPORTED;
}

int batch_common(const edt_batch_map_t* maps, int32_t n_maps, void* ws, size_t ws_bytes,
                 const edt_tuning_t* tuning, BatchPlan& p, EdtTuning& t)
{
    if (!maps || n_maps < 1 || n_maps > EDT_BATCH_MAX) {
        set_error("edt_compute_batched: need 1..%d maps, got %d", EDT_BATCH_MAX, n_maps);
        return EDT_ERR_ARG;
    }
    if (!ws || ws_bytes < edt_batch_workspace_bytes(n_maps)) {
        set_error("edt_compute_batched: workspace of %zu bytes is below %zu", ws_bytes,
                  edt_batch_workspace_bytes(n_maps));
        return EDT_ERR_WORKSPACE;
    }
    int nx = 0, ny = 0, nz = 0;
    for (int i = 0; i < n_maps; ++i) {
        nx = std::max(nx, maps[i].grid.nx);
        ny = std::max(ny, maps[i].grid.ny);
        nz = std::max(nz, maps[i].grid.nz);
    }
    const bool lean_ok = lean_batch_ok(maps, n_maps);
    if (tuning) {
        t.xy_tw = tuning->xy_tile;
        t.z_tw = tuning->z_tile;
        t.z_nt = 256;
        t.xy_nt = 256;
    } else {
        t = batch_current(n_maps, nx, ny, nz, lean_ok);
    }
    p.lean = t.xy_tw == LEAN_TILE && t.z_tw == LEAN_TILE;
    if (p.lean && !lean_ok) {
        set_error("edt_compute_batched: the lean tiles (64, 64) need every axis <= 512, rows of 64 voxels or "
                  "more, at most 256 rows and 128 slices");
        return EDT_ERR_UNSUPPORTED;
    }
    if (!p.lean && ((t.xy_tw != 16 && t.xy_tw != 32) || (t.z_tw != 16 && t.z_tw != 32 && t.z_tw != 64))) {
        set_error("edt_compute_batched: tiles (%d, %d) not available for batches", t.xy_tw, t.z_tw);
        return EDT_ERR_UNSUPPORTED;
    }
    // validates every map (the general plan's checks hold for lean batches too)
    int rc = make_plan(maps, n_maps, p.lean ? 32 : t.xy_tw, p.lean ? 64 : t.z_tw, p);
    if (rc) return rc;
    if (p.lean) return make_lean_plan(maps, n_maps, p.largs);
    constexpr size_t LDS_MAX = 160 * 1024 - 8192;
    if (xy_lds(t.xy_tw, p.ny_max) > LDS_MAX || z_lds(t.z_tw, p.nz_max) > LDS_MAX) {
        set_error("edt_compute_batched: tiles (%d, %d) need too much local memory", t.xy_tw, t.z_tw);
        return EDT_ERR_UNSUPPORTED;
    }
    return EDT_OK;
}

// ---------------------------------------------------------------------------
// Workspace of the allocation-free batched launch: the same words as a
// caller's workspace (queue head, error flag, one counter per map) for the
// largest batch, held by every GPU the library runs on for the life of the
// process.  Host code never passes the symbol itself to a kernel: it takes
// the array's device address on each device once, with that device current.
// ---------------------------------------------------------------------------
constexpr int SCRATCH_WORDS = 128;
static_assert(WS_DONE + 2 * EDT_BATCH_MAX <= SCRATCH_WORDS, "scratch too small for the largest batch");
static __device__ __align__(256) unsigned scratch[SCRATCH_WORDS];

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
unsigned* g_scratch_ptr[MAX_DEVICES] = {};

// The device address of scratch on the current device (looked up once per device).
int scratch_of_current_device(unsigned** out)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAX_DEVICES) {
        set_error("edt_compute_batched_noalloc: no usable current device (%d)", dev);
        return EDT_ERR_HIP;
    }
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) {
            set_error("edt_compute_batched_noalloc: hipGetSymbolAddress: %s", hipGetErrorString(e));
            return EDT_ERR_HIP;
        }
        g_scratch_ptr[dev] = static_cast<unsigned*>(ptr);
    }
    *out = g_scratch_ptr[dev];
    return EDT_OK;
}

}  // namespace

}  // namespace edtmi

using namespace edtmi;

extern "C" {

size_t edt_batch_workspace_bytes(int32_t n_maps)
{
    if (n_maps < 0) n_maps = 0;
    const size_t words = WS_DONE + 2 * (size_t)n_maps;
    return (words * 4 + 255) / 256 * 256;
}

int edt_compute_batched(const edt_batch_map_t* maps, int32_t n_maps, void* ws, size_t ws_bytes,
                        const edt_tuning_t* tuning, void* stream)
{
    BatchPlan p;
    EdtTuning t;
    int rc = batch_common(maps, n_maps, ws, ws_bytes, tuning, p, t);
    if (rc) return rc;
    return launch_batched(p, t.xy_tw, t.z_tw, static_cast<unsigned*>(ws), as_stream(stream));
}

int edt_compute_batched_noalloc(const edt_batch_map_t* maps, int32_t n_maps, const edt_tuning_t* tuning,
                                int32_t* timed_out, void* stream)
{
    unsigned* ws = nullptr;
    int rc = scratch_of_current_device(&ws);
    if (rc) return rc;
    BatchPlan p;
    EdtTuning t;
    rc = batch_common(maps, n_maps, ws, (size_t)SCRATCH_WORDS * sizeof(unsigned), tuning, p, t);
    if (rc) return rc;
    const hipStream_t st = as_stream(stream);
    rc = launch_batched(p, t.xy_tw, t.z_tw, ws, st);
    if (rc || !timed_out) return rc;
    hipLaunchKernelGGL(k_batch_flag_out, dim3(1), dim3(64), 0, st, ws, timed_out);
    return check_launch("k_batch_flag_out");
}

int edt_batch_status(const void* ws, int32_t* timed_out, void* stream)
{
    if (!ws || !timed_out) {
        set_error("edt_batch_status: NULL argument");
        return EDT_ERR_ARG;
    }
    unsigned flag = 0;
    const hipStream_t st = as_stream(stream);
    if (hipMemcpyAsync(&flag, static_cast<const unsigned*>(ws) + WS_ERR, sizeof(flag),
                       hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess) {
        set_error("edt_batch_status: copy failed");
        return EDT_ERR_HIP;
    }
    *timed_out = flag ? 1 : 0;
    return EDT_OK;
}

int edt_autotune_batched(const edt_batch_map_t* maps, int32_t n_maps, void* ws, size_t ws_bytes,
                         int32_t reps, edt_tuning_t* best, float* best_us, void* stream)
{
    if (reps < 1) {
        set_error("edt_autotune_batched: reps < 1");
        return EDT_ERR_ARG;
    }
    const hipStream_t st = as_stream(stream);
    const int XY[] = {16, 32, LEAN_TILE};   // (64, 64): the lean batch kernel
    const int Z[] = {16, 32, 64};
    float best_ms = 1e30f;
    EdtTuning bt{0, 0, 256};
    hipEvent_t a, b;
    if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) {
        set_error("edt_autotune_batched: hipEventCreate failed");
        return EDT_ERR_HIP;
    }
    int rc = EDT_OK;
    const bool lean_ok = lean_batch_ok(maps, n_maps);
    for (int txy : XY) {
        for (int tz : Z) {
            if (txy == LEAN_TILE && (tz != LEAN_TILE || !lean_ok)) continue;
            edt_tuning_t cand{txy, tz, 256};
            BatchPlan p;
            EdtTuning t;
            rc = batch_common(maps, n_maps, ws, ws_bytes, &cand, p, t);
            if (rc == EDT_ERR_UNSUPPORTED) {
                rc = EDT_OK;
                continue;
            }
            if (rc) break;
            float total = 0.0f;
            for (int r = 0; r <= reps && !rc; ++r) {
                (void)hipEventRecord(a, st);
                rc = launch_batched(p, txy, tz, static_cast<unsigned*>(ws), st);
                (void)hipEventRecord(b, st);
                if (rc) break;
                if (hipEventSynchronize(b) != hipSuccess) {
                    set_error("edt_autotune_batched: hipEventSynchronize failed");
                    rc = EDT_ERR_HIP;
                    break;
                }
                float ms = 0.0f;
                (void)hipEventElapsedTime(&ms, a, b);
                if (r > 0) total += ms;   // run 0 is a warm-up
            }
            if (rc) break;
            if (total / reps < best_ms) {
                best_ms = total / reps;
                bt = EdtTuning{txy, tz, 256, 256};
            }
        }
        if (rc) break;
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    if (rc) return rc;
    if (!bt.xy_tw) {
        set_error("edt_autotune_batched: no tile pair fits this batch");
        return EDT_ERR_UNSUPPORTED;
    }
    int nx = 0, ny = 0, nz = 0;
    for (int i = 0; i < n_maps; ++i) {
        nx = std::max(nx, maps[i].grid.nx);
        ny = std::max(ny, maps[i].grid.ny);
        nz = std::max(nz, maps[i].grid.nz);
    }
    tuned_store(1, n_maps, nx, ny, nz, bt);
    if (best) {
        best->xy_tile = bt.xy_tw;
        best->z_tile = bt.z_tw;
        best->z_group = 256;
        best->xy_group = 256;
    }
    if (best_us) *best_us = 1000.0f * best_ms;
    // leave the chosen tiling's result in the outputs
    BatchPlan p;
    EdtTuning t;
    edt_tuning_t chosen{bt.xy_tw, bt.z_tw, 256};
    rc = batch_common(maps, n_maps, ws, ws_bytes, &chosen, p, t);
    if (!rc) rc = launch_batched(p, bt.xy_tw, bt.z_tw, static_cast<unsigned*>(ws), st);
    if (!rc && hipStreamSynchronize(st) != hipSuccess) {
        set_error("edt_autotune_batched: stream synchronisation failed");
        rc = EDT_ERR_HIP;
    }
    return rc;
}

}  // extern "C"
