// Autotuner of the EDT tile widths (the band parameters of Alg. 1).
//
// Every valid (xy_tile, z_tile) pair is timed on a representative map with
// HIP events; the pass times are independent, so the best pair is the best
// xy tile with the best z tile.  The winner is cached per grid shape for the
// life of the process and used by edt_compute.
#include <map>
#include <mutex>
#include <tuple>

#include "common.h"

namespace edtmi {

namespace {
std::mutex g_tune_mu;
std::map<std::tuple<int, int, int>, EdtTuning> g_tuned;

const int XY_TILES[] = {16, 32, 64};
const int XY_GROUPS[] = {256, 512};
const int Z_TILES[] = {8, 16, 32, 64};
const int Z_GROUPS[] = {64, 128, 256, 512};

// Average time (ms) of `reps` launches of one pass with tile tw.
int time_pass(const edt_grid_t* g, const uint8_t* occ, int32_t* d2, int32_t* site, int pass,
              int tw, int nt, int reps, hipStream_t st, float* ms)
{
    hipEvent_t a, b;
    if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) {
        set_error("edt_autotune: hipEventCreate failed");
        return EDT_ERR_HIP;
    }
    int rc = EDT_OK;
    const EdtTuning prep = current_tuning(g);
    float total = 0.0f;
    // iteration 0 is an untimed warm-up
    for (int r = 0; r <= reps && !rc; ++r) {
        // the z pass consumes its input in place: give it a fresh xy result
        if (pass == 2)
            rc = launch_edt_xy(g, occ, d2, reinterpret_cast<uint32_t*>(site), prep.xy_tw, prep.xy_nt, st);
        if (rc) break;
        (void)hipEventRecord(a, st);
        rc = pass == 1 ? launch_edt_xy(g, occ, d2, reinterpret_cast<uint32_t*>(site), tw, nt, st)
                       : launch_edt_z(g, d2, site, tw, nt, st);
        (void)hipEventRecord(b, st);
        if (rc) break;
        if (hipEventSynchronize(b) != hipSuccess) {
            set_error("edt_autotune: hipEventSynchronize failed");
            rc = EDT_ERR_HIP;
            break;
        }
        float ms1 = 0.0f;
        (void)hipEventElapsedTime(&ms1, a, b);
        if (r > 0) total += ms1;
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    *ms = reps > 0 ? total / reps : 0.0f;
    return rc;
}
}  // namespace

EdtTuning current_tuning(const edt_grid_t* g)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tuned.find(std::make_tuple(g->nx, g->ny, g->nz));
    return it != g_tuned.end() ? it->second : default_tuning(g);
}

}  // namespace edtmi

using namespace edtmi;

extern "C" {

int edt_default_tuning(const edt_grid_t* grid, edt_tuning_t* out)
{
    int rc = check_grid(grid);
    if (rc) return rc;
    if (!out) {
        set_error("edt_default_tuning: out is NULL");
        return EDT_ERR_ARG;
    }
    const EdtTuning t = current_tuning(grid);
    out->xy_tile = t.xy_tw;
    out->z_tile = t.z_tw;
    out->z_group = t.z_nt;
    out->xy_group = t.xy_nt;
    return EDT_OK;
}

int edt_autotune(const edt_grid_t* grid, const uint8_t* occ, int32_t* d2, int32_t* site,
                 int32_t reps, edt_tuning_t* best, float* best_us, void* stream)
{
    int rc = check_grid(grid);
    if (rc) return rc;
    if (!occ || !d2 || !site || reps < 1) {
        set_error("edt_autotune: NULL buffer or reps < 1");
        return EDT_ERR_ARG;
    }
    const hipStream_t st = as_stream(stream);
    float best_xy = 1e30f, best_z = 1e30f;
    int bxy = 0, bxnt = 0, bz = 0, bnt = 0;
    for (int nt : XY_GROUPS) {
        for (int tw : XY_TILES) {
            if (!tile_ok(1, tw, grid, nt)) continue;
            float ms = 0.0f;
            rc = time_pass(grid, occ, d2, site, 1, tw, nt, reps, st, &ms);
            if (rc) return rc;
            if (ms < best_xy) { best_xy = ms; bxy = tw; bxnt = nt; }
        }
    }
    for (int nt : Z_GROUPS) {
        for (int tw : Z_TILES) {
            if (!tile_ok(2, tw, grid, nt)) continue;
            float ms = 0.0f;
            rc = time_pass(grid, occ, d2, site, 2, tw, nt, reps, st, &ms);
            if (rc) return rc;
            if (ms < best_z) { best_z = ms; bz = tw; bnt = nt; }
        }
    }
    if (!bxy || !bz) {
        set_error("edt_autotune: no valid tile for this grid");
        return EDT_ERR_UNSUPPORTED;
    }
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tuned[std::make_tuple(grid->nx, grid->ny, grid->nz)] = EdtTuning{bxy, bz, bnt, bxnt};
    }
    // leave a complete transform in d2 / site
    rc = launch_edt_xy(grid, occ, d2, reinterpret_cast<uint32_t*>(site), bxy, bxnt, st);
    if (!rc) rc = launch_edt_z(grid, d2, site, bz, bnt, st);
    if (rc) return rc;
    if (hipStreamSynchronize(st) != hipSuccess) {
        set_error("edt_autotune: stream synchronisation failed");
        return EDT_ERR_HIP;
    }
    if (best) {
        best->xy_tile = bxy;
        best->z_tile = bz;
        best->z_group = bnt;
        best->xy_group = bxnt;
    }
    if (best_us) *best_us = 1000.0f * (best_xy + best_z);
    return EDT_OK;
}

}  // extern "C"
