// The exact squared EDT on gfx950 for one map: the xy-tile kernel (steps 1-3
// of Sec. III-C in every slice) and the z-tile kernel (step 4), their
// launchers and the tile heuristics.  The tile code is in edt_tiles.h (every
// shape and tiling) and edt_lean.h (the 64-column tiles of maps up to 256 rows
// and 128 slices).
#include <algorithm>

#include "edt_lean.h"

namespace edtmi {

namespace {

using namespace tiles;

// Map of launch tile T (the maps' tile ranges are consecutive).
__device__ __forceinline__ int map_of(const EdtMapSet& s, int T)
{
    int m = 0;
    while (m + 1 < s.n && s.m[m + 1].begin <= T) ++m;
    return __builtin_amdgcn_readfirstlane(m);
}

// True while the map's gate (if any) holds 0: its work-groups return at once.
__device__ __forceinline__ bool gated_off(const EdtMap& d)
{
    return d.gate && __builtin_amdgcn_readfirstlane(*d.gate) == 0;
}

template <int TW, bool WIDE, int NTX>
__global__ __launch_bounds__(NTX) void k_edt_xy(EdtMapSet s)
{
    extern __shared__ uint32_t lds[];
    // the tiles of a slice read the same occupancy bytes: chunks of 16 tiles
    // (one or two slices) share an XCD's L2, and the slices, whose work is
    // very uneven, rotate over the XCDs
    const int T = xcd_chunk_remap(blockIdx.x, s.total, 16);
    const EdtMap& d = s.m[map_of(s, T)];
    if (gated_off(d)) return;
    edt_xy_tile<TW, WIDE, NTX>(d.occ, reinterpret_cast<uint32_t*>(d.site), d.nx, d.ny, d.nz, d.ntx,
                               T - d.begin, lds);
}

// Row records (step 1) of every map of the set: each wave takes
// record_rows_per_wave(nx) whole rows of one map, four waves per work-group;
// s.m[i].begin is the map's first wave.
__global__ __launch_bounds__(256) void k_row_records(EdtMapSet s)
{
    const int wv = __builtin_amdgcn_readfirstlane((int)blockIdx.x * 4 + (int)(threadIdx.x >> 6));
    if (wv >= s.total) return;
    const EdtMap& d = s.m[map_of(s, wv)];
    if (gated_off(d)) return;
    const int per = record_rows_per_wave(d.occ, d.nx);
    const int row0 = (wv - d.begin) * per;
    const int nrows = min(per, d.ny * d.nz - row0);
    if (record_words(d.occ, d.nx))
        row_summary_words(d.occ, d.nx, (size_t)row0, nrows, row_records(d.d2, d.nx, d.ny, d.nz));
    else
        row_summary(d.occ, d.nx, (size_t)row0, nrows, row_records(d.d2, d.nx, d.ny, d.nz));
}

// Steps 2-3 from the row records.
template <int TW, bool WIDE, int NTX>
__global__ __launch_bounds__(NTX) void k_edt_xy_rows(EdtMapSet s)
{
    extern __shared__ uint32_t lds[];
    // as in k_edt_xy: chunks of 16 tiles per XCD, rotating over the XCDs
    const int T = xcd_chunk_remap(blockIdx.x, s.total, 16);
    const EdtMap& d = s.m[map_of(s, T)];
    if (gated_off(d)) return;
    edt_xy_tile_rows<TW, WIDE, NTX>(row_records(d.d2, d.nx, d.ny, d.nz), reinterpret_cast<uint32_t*>(d.site),
                                    d.nx, d.ny, d.ntx, T - d.begin, lds);
}

template <int TW, bool WIDE, int NTZ>
__global__ __launch_bounds__(NTZ) void k_edt_z(EdtMapSet s)
{
    extern __shared__ uint32_t lds[];
    // tiles narrower than 64 columns share cache lines with their neighbours:
    // the tiles of 64 columns of a row stay on one XCD, and rows (whose work
    // is very uneven) rotate over all eight
    const int T = TW >= 64 ? (int)blockIdx.x : xcd_chunk_remap(blockIdx.x, s.total, 64 / TW);
    const EdtMap& d = s.m[map_of(s, T)];
    if (gated_off(d)) return;
    edt_z_tile<TW, WIDE, NTZ>(d.d2, d.site, d.nx, d.ny, d.nz, d.ntx, T - d.begin, lds);
}

// Lean tiles (edt_lean.h): 64 columns, one wave per band.
__global__ __launch_bounds__(256) void k_edt_z_lean(EdtMapSet s)
{
    const int T = (int)blockIdx.x;
    const EdtMap& d = s.m[map_of(s, T)];
    if (gated_off(d)) return;
    __shared__ lean::ZLds lds;
    lean::z_tile(d.d2, d.site, d.nx, d.ny, d.nz, d.ntx, T - d.begin, (int)threadIdx.x, lds);
}

// Ent = uint16_t (narrow stack entries) when every map has at most 256 columns.
template <typename Ent>
__global__ __launch_bounds__(512) void k_edt_xy_lean(EdtMapSet s)
{
    // as in k_edt_xy: chunks of 16 tiles per XCD, rotating over the XCDs
    const int T = xcd_chunk_remap(blockIdx.x, s.total, 16);
    const EdtMap& d = s.m[map_of(s, T)];
    if (gated_off(d)) return;
    __shared__ lean::XyLdsT<Ent> lds;
    lean::xy_tile<Ent>(row_records(d.d2, d.nx, d.ny, d.nz), reinterpret_cast<uint32_t*>(d.site), d.nx, d.ny,
                       d.ntx, T - d.begin, lds);
}

// Allow dynamic LDS beyond the 64 KiB default (gfx950 has 160 KiB per
// work-group); once per kernel instantiation.
template <typename K>
int allow_lds(K kernel, bool& done)
{
    if (done) return EDT_OK;
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024 - 8192);
    if (e != hipSuccess) {
        set_error("hipFuncSetAttribute: %s", hipGetErrorString(e));
        return EDT_ERR_HIP;
    }
    done = true;
    return EDT_OK;
}

// Step 1 once per row when every map's rows are at least 256 voxels long,
// else inside every tile from the slice.  The records need rows of 64 or more
// to fit in d2; below 256 a slice is staged by few tiles, and the extra
// kernel costs more than the staging it saves (measured on maps of 64-256).
bool rows_first(const EdtMapSet& s)
{
    for (int i = 0; i < s.n; ++i)
        if (s.m[i].nx < 256 || !s.m[i].d2) return false;
    return true;
}

// The lean tiles take maps with every axis <= 512 (24-bit arithmetic), up to
// 256 rows (xy) or 128 slices (z), and rows of 64 voxels or more (the row
// records must fit into d2).
bool lean_xy_ok(const EdtMapSet& s)
{
    if (s.wide) return false;
    for (int i = 0; i < s.n; ++i)
        if (s.m[i].ny > lean::XY_MAX || s.m[i].nx < 64 || !s.m[i].d2) return false;
    return true;
}

bool lean_z_ok(const EdtMapSet& s) { return !s.wide && s.nz_max <= lean::Z_MAX; }

// Step 1 of every map of the set once per row, into the maps' d2 buffers.
int launch_row_records(const EdtMapSet& s, hipStream_t st)
{
    static thread_local EdtMapSet r;   // the maps counted in waves (2.3 KiB: off the stack)
    r = s;
    int waves = 0;
    for (int i = 0; i < s.n; ++i) {
        const int per = record_rows_per_wave(s.m[i].occ, s.m[i].nx);
        r.m[i].begin = waves;
        waves += (s.m[i].ny * s.m[i].nz + per - 1) / per;
    }
    r.total = waves;
    hipLaunchKernelGGL(k_row_records, dim3((waves + 3) / 4), dim3(256), 0, st, r);
    return check_launch("k_row_records");
}

template <int TW, bool WIDE, int NTX>
int launch_xy_w(const EdtMapSet& s, hipStream_t st)
{
    if (TW == 64 && NTX == 512 && !WIDE && lean_xy_ok(s)) {
        int rc = launch_row_records(s, st);
        if (rc) return rc;
        // narrow stack entries (maps of at most 256 columns) fit twice the
        // work-groups per CU but cost a little more per tile: they pay only
        // when the launch has more tiles than the wide ones keep resident
        // (2 per CU)
        static int n_cu = 0;
        if (!n_cu) {
            int dev = 0, c = 0;
            if (hipGetDevice(&dev) == hipSuccess &&
                hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && c > 0)
                n_cu = c;
            else
                n_cu = 256;
        }
        int nx_max = 0;
        for (int i = 0; i < s.n; ++i) nx_max = std::max(nx_max, s.m[i].nx);
        if (nx_max <= 256 && s.total > 2 * n_cu)
            hipLaunchKernelGGL(k_edt_xy_lean<uint16_t>, dim3(s.total), dim3(512), 0, st, s);
        else
            hipLaunchKernelGGL(k_edt_xy_lean<uint32_t>, dim3(s.total), dim3(512), 0, st, s);
        return check_launch("k_edt_xy_lean");
    }
    if (rows_first(s)) {
        int rc = launch_row_records(s, st);
        if (rc) return rc;
        static bool done_rows = false;
        rc = allow_lds(k_edt_xy_rows<TW, WIDE, NTX>, done_rows);
        if (rc) return rc;
        hipLaunchKernelGGL((k_edt_xy_rows<TW, WIDE, NTX>), dim3(s.total), dim3(NTX),
                           xy_rows_lds(TW, s.ny_max, NTX), st, s);
        return check_launch("k_edt_xy_rows");
    }
    static bool done = false;
    int rc = allow_lds(k_edt_xy<TW, WIDE, NTX>, done);
    if (rc) return rc;
    hipLaunchKernelGGL((k_edt_xy<TW, WIDE, NTX>), dim3(s.total), dim3(NTX), xy_lds(TW, s.ny_max, NTX),
                       st, s);
    return check_launch("k_edt_xy");
}

template <int TW, int NTX>
int launch_xy_tw(const EdtMapSet& s, hipStream_t st)
{
    return s.wide ? launch_xy_w<TW, true, NTX>(s, st) : launch_xy_w<TW, false, NTX>(s, st);
}

template <int TW, bool WIDE, int NTZ>
int launch_z_t(const EdtMapSet& s, hipStream_t st)
{
    if (TW == 64 && NTZ == 256 && !WIDE && lean_z_ok(s)) {
        hipLaunchKernelGGL(k_edt_z_lean, dim3(s.total), dim3(64 * ((s.nz_max + 31) / 32)), 0, st, s);
        return check_launch("k_edt_z_lean");
    }
    static bool done = false;
    int rc = allow_lds(k_edt_z<TW, WIDE, NTZ>, done);
    if (rc) return rc;
    hipLaunchKernelGGL((k_edt_z<TW, WIDE, NTZ>), dim3(s.total), dim3(NTZ), z_lds(TW, s.nz_max, NTZ), st,
                       s);
    return check_launch("k_edt_z");
}

template <int TW, int NTZ>
int launch_z_tw(const EdtMapSet& s, hipStream_t st)
{
    return s.wide ? launch_z_t<TW, true, NTZ>(s, st) : launch_z_t<TW, false, NTZ>(s, st);
}

// The tiles of every map of the set, ntx column tiles of width tw per row
// of the pass (rows: z slices for xy, y rows for z).
void fill_set(const edt_batch_map_t* maps, int n, int tw, bool z_pass, EdtMapSet& s,
              const int* gates)
{
    s.n = n;
    s.total = 0;
    s.ny_max = s.nz_max = 0;
    s.wide = false;
    for (int i = 0; i < n; ++i) {
        const edt_grid_t& g = maps[i].grid;
        EdtMap& d = s.m[i];
        d.occ = maps[i].occ;
        d.d2 = maps[i].d2;
        d.site = maps[i].site;
        d.nx = g.nx;
        d.ny = g.ny;
        d.nz = g.nz;
        d.ntx = (g.nx + tw - 1) / tw;
        d.begin = s.total;
        d.gate = gates ? gates + i : nullptr;
        s.total += (z_pass ? g.ny : g.nz) * d.ntx;
        s.ny_max = std::max(s.ny_max, g.ny);
        s.nz_max = std::max(s.nz_max, g.nz);
        s.wide = s.wide || needs_wide(&g);
    }
}

}  // namespace

// Every cross product of the dominance test stays below 2^31 when each axis
// has at most 512 voxels; larger grids use 64-bit products.
bool needs_wide(const edt_grid_t* g) { return g->nx > 512 || g->ny > 512 || g->nz > 512; }

bool tile_ok(int pass, int tw, const edt_grid_t* g, int nt)
{
    constexpr size_t LDS_MAX = 160 * 1024 - 8192;
    if (pass == 1) {
        if (tw != 16 && tw != 32 && tw != 64) return false;
        if (nt != 64 && nt != 128 && nt != 256 && !(nt == 512 && tw >= 32)) return false;
        if (tw > nt) return false;
        return xy_lds(tw, g->ny, nt) <= LDS_MAX;
    }
    if (tw != 8 && tw != 16 && tw != 32 && tw != 64) return false;
    if (nt != 64 && nt != 128 && nt != 256 && !(nt == 512 && tw == 64)) return false;
    if (tw > nt) return false;
    return z_lds(tw, g->nz, nt) <= LDS_MAX;
}

EdtTuning default_tuning(const edt_grid_t* g)
{
    // measured on MI355X: 32-wide xy tiles up to 256 rows; up to 512 rows the
    // same tiles with 512 threads (32 rows per band, and each slice staged by
    // half as many work-groups as with 16-wide tiles); 16-wide beyond.  z
    // tiles keep about 32 positions per band
    EdtTuning t;
    t.xy_tw = g->ny <= 512 ? 32 : 16;
    t.xy_nt = g->ny > 256 && g->ny <= 512 ? 512 : 256;
    // with more than 256 slices as well there are tiles enough to balance:
    // 16-wide tiles in 256-thread work-groups (512^3 blobs: 919 against
    // 1006 us for 32 / 512)
    if (g->ny > 256 && g->nz > 256) {
        t.xy_tw = 16;
        t.xy_nt = 256;
    }
    t.z_tw = g->nz <= 128 ? 64 : (g->nz <= 256 ? 32 : 16);
    t.z_nt = 256;
    // the lean tiles where they apply (64 / 512 for xy, 64 / 256 for z)
    if (!needs_wide(g) && g->ny <= lean::XY_MAX && g->nx >= 64) {
        t.xy_tw = 64;
        t.xy_nt = 512;
    }
    if (!tile_ok(1, t.xy_tw, g, t.xy_nt)) {
        t.xy_tw = 16;
        t.xy_nt = 256;
    }
    if (!tile_ok(2, t.z_tw, g, t.z_nt)) t.z_tw = 8;
    return t;
}

int make_map_sets(const edt_batch_map_t* maps, int n, const EdtTuning& t, EdtMapSet& xy,
                  EdtMapSet& z, const int* gates)
{
    if (!maps || n < 1 || n > EDT_BATCH_MAX) {
        set_error("need 1..%d maps, got %d", EDT_BATCH_MAX, n);
        return EDT_ERR_ARG;
    }
    edt_grid_t big{};
    big.voxel = 1.0f;
    for (int i = 0; i < n; ++i) {
        const edt_grid_t* g = &maps[i].grid;
        int rc = check_grid(g);
        if (rc) return rc;
        if (!maps[i].occ || !maps[i].d2 || !maps[i].site) {
            set_error("map %d: NULL occ, d2 or site", i);
            return EDT_ERR_ARG;
        }
        big.nx = std::max(big.nx, g->nx);
        big.ny = std::max(big.ny, g->ny);
        big.nz = std::max(big.nz, g->nz);
    }
    if (!tile_ok(1, t.xy_tw, &big, t.xy_nt) || !tile_ok(2, t.z_tw, &big, t.z_nt)) {
        set_error("tiles (%d / %d, %d / %d) not valid for maps up to %d x %d x %d", t.xy_tw, t.xy_nt,
                  t.z_tw, t.z_nt, big.nx, big.ny, big.nz);
        return EDT_ERR_UNSUPPORTED;
    }
    fill_set(maps, n, t.xy_tw, false, xy, gates);
    fill_set(maps, n, t.z_tw, true, z, gates);
    return EDT_OK;
}

int launch_edt_xy_set(const EdtMapSet& s, int tw, int nt, hipStream_t st)
{
    if (nt == 512) {
        switch (tw) {
            case 64: return launch_xy_tw<64, 512>(s, st);
            case 32: return launch_xy_tw<32, 512>(s, st);
        }
    } else if (nt == 256) {
        switch (tw) {
            case 64: return launch_xy_tw<64, 256>(s, st);
            case 32: return launch_xy_tw<32, 256>(s, st);
            case 16: return launch_xy_tw<16, 256>(s, st);
        }
    } else if (nt == 128) {
        switch (tw) {
            case 64: return launch_xy_tw<64, 128>(s, st);
            case 32: return launch_xy_tw<32, 128>(s, st);
            case 16: return launch_xy_tw<16, 128>(s, st);
        }
    } else if (nt == 64) {
        switch (tw) {
            case 64: return launch_xy_tw<64, 64>(s, st);
            case 32: return launch_xy_tw<32, 64>(s, st);
            case 16: return launch_xy_tw<16, 64>(s, st);
        }
    }
    set_error("bad xy tile %d / group %d", tw, nt);
    return EDT_ERR_ARG;
}

int launch_edt_z_set(const EdtMapSet& s, int tw, int nt, hipStream_t st)
{
    if (nt == 512 && tw == 64) return launch_z_tw<64, 512>(s, st);
    if (nt == 256) {
        switch (tw) {
            case 64: return launch_z_tw<64, 256>(s, st);
            case 32: return launch_z_tw<32, 256>(s, st);
            case 16: return launch_z_tw<16, 256>(s, st);
            case 8: return launch_z_tw<8, 256>(s, st);
        }
    } else if (nt == 128) {
        switch (tw) {
            case 64: return launch_z_tw<64, 128>(s, st);
            case 32: return launch_z_tw<32, 128>(s, st);
            case 16: return launch_z_tw<16, 128>(s, st);
            case 8: return launch_z_tw<8, 128>(s, st);
        }
    } else if (nt == 64) {
        switch (tw) {
            case 64: return launch_z_tw<64, 64>(s, st);
            case 32: return launch_z_tw<32, 64>(s, st);
            case 16: return launch_z_tw<16, 64>(s, st);
            case 8: return launch_z_tw<8, 64>(s, st);
        }
    }
    set_error("bad z tile %d / group %d", tw, nt);
    return EDT_ERR_ARG;
}

namespace {
edt_batch_map_t one_map(const edt_grid_t* g, const uint8_t* occ, int32_t* d2, int32_t* site)
{
    edt_batch_map_t m{};
    m.grid = *g;
    m.occ = occ;
    m.d2 = d2;
    m.site = site;
    return m;
}
}  // namespace

int launch_edt_xy(const edt_grid_t* g, const uint8_t* occ, int32_t* d2, uint32_t* xy, int tw, int nt,
                  hipStream_t st, const int* gate)
{
    const edt_batch_map_t m = one_map(g, occ, d2, reinterpret_cast<int32_t*>(xy));
    EdtMapSet s;
    fill_set(&m, 1, tw, false, s, gate);
    return launch_edt_xy_set(s, tw, nt, st);
}

int launch_edt_z(const edt_grid_t* g, int32_t* d2, int32_t* site, int tw, int nt, hipStream_t st,
                 const int* gate)
{
    const edt_batch_map_t m = one_map(g, nullptr, d2, site);
    EdtMapSet s;
    fill_set(&m, 1, tw, true, s, gate);
    return launch_edt_z_set(s, tw, nt, st);
}

}  // namespace edtmi
