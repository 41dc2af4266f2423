// Internal helpers shared by the library's translation units (not exported).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <string>

#include "edt.h"

namespace edtmi {

// Last error message of the calling thread.
void set_error(const char* fmt, ...);
void clear_error();

inline hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

// Validates a grid; sets the error message and returns a status.
int check_grid(const edt_grid_t* g);

inline int64_t grid_voxels(const edt_grid_t* g)
{
    return (int64_t)g->nx * g->ny * g->nz;
}

// Checks the launch that was just enqueued.
inline int check_launch(const char* what)
{
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        set_error("%s: launch failed: %s", what, hipGetErrorString(e));
        return EDT_ERR_HIP;
    }
    return EDT_OK;
}

// Tile widths (columns per work-group) of the two EDT passes; each
// work-group has 256 threads, so a column gets 256 / tile bands.
struct EdtTuning {
    int xy_tw;
    int z_tw;
    int z_nt;   // threads per z work-group (64, 128 or 256)
    int xy_nt;  // threads per xy work-group (64, 128 or 256)
};
// The tiles an API tuning struct asks for (0 group sizes mean 256).
inline EdtTuning tuning_from(const edt_tuning_t* p)
{
    EdtTuning t;
    t.xy_tw = p->xy_tile;
    t.z_tw = p->z_tile;
    t.z_nt = p->z_group ? p->z_group : 256;
    t.xy_nt = p->xy_group ? p->xy_group : 256;
    return t;
}
EdtTuning default_tuning(const edt_grid_t* g);   // heuristic
EdtTuning current_tuning(const edt_grid_t* g);   // autotuned if cached, else heuristic
// The autotuners' choices, per device architecture: single maps (kind 0) by
// (nx, ny, nz), batches (kind 1) by (maps, largest nx, ny, nz).  Lookups
// and stores use the current device's architecture.
bool tuned_lookup(int kind, int n, int nx, int ny, int nz, EdtTuning& out);
void tuned_store(int kind, int n, int nx, int ny, int nz, const EdtTuning& t);
bool tile_ok(int pass, int tw, const edt_grid_t* g, int nt);   // pass 1 = xy, 2 = z
bool needs_wide(const edt_grid_t* g);
// The xy pass of one map into xy (the site buffer); d2 may serve as scratch.
int launch_edt_xy(const edt_grid_t* g, const uint8_t* occ, int32_t* d2, uint32_t* xy, int tw, int nt,
                  hipStream_t st, const int* gate = nullptr);
int launch_edt_z(const edt_grid_t* g, int32_t* d2, int32_t* site, int tw, int nt, hipStream_t st,
                 const int* gate = nullptr);

// One launch per pass over the tiles of several maps: tile T of the launch
// belongs to the map whose [begin, begin + tiles) holds it.  Passed by value
// as the kernel argument (about 2.3 KiB).
struct EdtMap {
    const uint8_t* occ;
    int32_t* d2;
    int32_t* site;   // the packed 2D sites between the passes
    int nx, ny, nz;
    int ntx;         // column tiles per row of this pass
    int begin;       // first tile of this map in the launch
    const int* gate; // nullable: this map's work-groups do nothing while *gate == 0
};
struct EdtMapSet {
    int n;
    int total;       // tiles of all maps
    int ny_max, nz_max;
    bool wide;
    EdtMap m[EDT_BATCH_MAX];
};
// Validates the maps and the tiles and fills the two passes' sets; gates
// (nullable, device int [n]) switch maps off from the device.
int make_map_sets(const edt_batch_map_t* maps, int n, const EdtTuning& t, EdtMapSet& xy,
                  EdtMapSet& z, const int* gates = nullptr);
int launch_edt_xy_set(const EdtMapSet& s, int tw, int nt, hipStream_t st);
int launch_edt_z_set(const EdtMapSet& s, int tw, int nt, hipStream_t st);

// Work-group index remap: chunks of C consecutive logical tiles each land on
// one XCD (the dispatcher deals work-groups to the 8 XCDs round-robin), and
// consecutive chunks go to consecutive XCDs, so neighbouring tiles share an
// L2 while uneven work spreads over all eight.  A bijection of [0, G): the
// tail that does not fill 8 whole chunks keeps launch order.
__device__ inline int xcd_chunk_remap(int b, int G, int C)
{
    const int full = G / (8 * C) * (8 * C);
    if (b >= full) return b;
    const int xcd = b & 7, k = b >> 3;
    return (k / C) * 8 * C + xcd * C + k % C;
}

}  // namespace edtmi
