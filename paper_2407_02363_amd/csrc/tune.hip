// Autotuner of the EDT tile widths (the band parameters of Alg. 1), and the
// cache of its choices.
//
// Every valid (xy_tile, z_tile) pair is timed on a representative map with
// HIP events; the pass times are independent, so the best pair is the best
// xy tile with the best z tile.  The winner is cached per device
// architecture and grid shape and used by edt_compute; the cache can be
// written to a text file and read back by a later process.
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "common.h"

namespace edtmi {

namespace {
// (architecture, kind, maps, nx, ny, nz) -> tiles
using TuneKey = std::tuple<std::string, int, int, int, int, int>;
std::mutex g_tune_mu;
std::map<TuneKey, EdtTuning> g_tuned;

// The current device's architecture name without its feature suffixes
// ("gfx950"), "" when there is no device.
std::string current_arch()
{
    constexpr int MAX_DEV = 64;
    static std::string names[MAX_DEV];
    static std::once_flag once[MAX_DEV];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAX_DEV) return std::string();
    std::call_once(once[dev], [dev]() {
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, dev) == hipSuccess) {
            std::string a = prop.gcnArchName;
            names[dev] = a.substr(0, a.find(':'));
        }
    });
    return names[dev];
}

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

bool tuned_lookup(int kind, int n, int nx, int ny, int nz, EdtTuning& out)
{
    const std::string arch = current_arch();
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tuned.find(TuneKey{arch, kind, n, nx, ny, nz});
    if (it == g_tuned.end()) return false;
    out = it->second;
    return true;
}

void tuned_store(int kind, int n, int nx, int ny, int nz, const EdtTuning& t)
{
    const std::string arch = current_arch();
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tuned[TuneKey{arch, kind, n, nx, ny, nz}] = t;
}

EdtTuning current_tuning(const edt_grid_t* g)
{
    EdtTuning t;
    return tuned_lookup(0, 0, g->nx, g->ny, g->nz, t) ? t : default_tuning(g);
}

namespace {
constexpr const char* CACHE_HEADER = "edtmi tuning cache v1";

// A cache line's tiles are ones the library can launch for its shape.
bool entry_ok(int kind, int n, int nx, int ny, int nz, const EdtTuning& t)
{
    edt_grid_t g{nx, ny, nz, {0.0f, 0.0f, 0.0f}, 1.0f};
    if (check_grid(&g)) return false;
    if (kind == 0) return n == 0 && tile_ok(1, t.xy_tw, &g, t.xy_nt) && tile_ok(2, t.z_tw, &g, t.z_nt);
    const bool lean = t.xy_tw == 64 && t.z_tw == 64;   // the lean batch kernel
    return n >= 1 && n <= EDT_BATCH_MAX && (lean || ((t.xy_tw == 16 || t.xy_tw == 32) &&
           (t.z_tw == 16 || t.z_tw == 32 || t.z_tw == 64))) && t.xy_nt == 256 && t.z_nt == 256;
}
}  // namespace

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
    tuned_store(0, 0, grid->nx, grid->ny, grid->nz, EdtTuning{bxy, bz, bnt, bxnt});
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

int edt_tuning_cache_save(const char* path)
{
    if (!path) {
        set_error("edt_tuning_cache_save: path is NULL");
        return EDT_ERR_ARG;
    }
    std::vector<std::pair<TuneKey, EdtTuning>> all;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        all.assign(g_tuned.begin(), g_tuned.end());
    }
    FILE* f = std::fopen(path, "w");
    if (!f) {
        set_error("edt_tuning_cache_save: cannot open %s for writing", path);
        return EDT_ERR_ARG;
    }
    std::fprintf(f, "%s\n", CACHE_HEADER);
    for (const auto& e : all) {
        const TuneKey& k = e.first;
        const EdtTuning& t = e.second;
        if (std::get<1>(k) == 0)
            std::fprintf(f, "single %s %d %d %d xy %d %d z %d %d\n", std::get<0>(k).c_str(), std::get<3>(k),
                         std::get<4>(k), std::get<5>(k), t.xy_tw, t.xy_nt, t.z_tw, t.z_nt);
        else
            std::fprintf(f, "batch %s %d %d %d %d xy %d %d z %d %d\n", std::get<0>(k).c_str(), std::get<2>(k),
                         std::get<3>(k), std::get<4>(k), std::get<5>(k), t.xy_tw, t.xy_nt, t.z_tw, t.z_nt);
    }
    const bool ok = std::fflush(f) == 0;
    std::fclose(f);
    if (!ok) {
        set_error("edt_tuning_cache_save: writing %s failed", path);
        return EDT_ERR_ARG;
    }
    return (int)all.size();
}

int edt_tuning_cache_load(const char* path)
{
    if (!path) {
        set_error("edt_tuning_cache_load: path is NULL");
        return EDT_ERR_ARG;
    }
    FILE* f = std::fopen(path, "r");
    if (!f) {
        set_error("edt_tuning_cache_load: cannot open %s", path);
        return EDT_ERR_ARG;
    }
    std::vector<std::pair<TuneKey, EdtTuning>> got;
    char line[512];
    int lineno = 0, rc = EDT_OK;
    while (std::fgets(line, sizeof line, f)) {
        ++lineno;
        const size_t len = std::strlen(line);
        if (len + 1 == sizeof line && line[len - 1] != '\n') {
            set_error("edt_tuning_cache_load: %s:%d: line too long", path, lineno);
            rc = EDT_ERR_ARG;
            break;
        }
        if (lineno == 1) {
            if (std::strncmp(line, CACHE_HEADER, std::strlen(CACHE_HEADER)) != 0) {
                set_error("edt_tuning_cache_load: %s is not a tuning cache (first line)", path);
                rc = EDT_ERR_ARG;
                break;
            }
            continue;
        }
        if (line[0] == '\n' || line[0] == '#') continue;
        char kind[16] = "", arch[64] = "";
        int n = 0, nx, ny, nz, consumed = 0;
        EdtTuning t{};
        bool ok = false;
        if (std::sscanf(line, "%15s %63s", kind, arch) == 2) {
            if (!std::strcmp(kind, "single"))
                ok = std::sscanf(line, "single %*s %d %d %d xy %d %d z %d %d %n", &nx, &ny, &nz, &t.xy_tw,
                                 &t.xy_nt, &t.z_tw, &t.z_nt, &consumed) == 7;
            else if (!std::strcmp(kind, "batch"))
                ok = std::sscanf(line, "batch %*s %d %d %d %d xy %d %d z %d %d %n", &n, &nx, &ny, &nz,
                                 &t.xy_tw, &t.xy_nt, &t.z_tw, &t.z_nt, &consumed) == 8;
        }
        const int k = !std::strcmp(kind, "batch") ? 1 : 0;
        if (!ok || line[consumed] != '\0' || !entry_ok(k, n, nx, ny, nz, t)) {
            set_error("edt_tuning_cache_load: %s:%d: not a valid entry", path, lineno);
            rc = EDT_ERR_ARG;
            break;
        }
        got.emplace_back(TuneKey{arch, k, n, nx, ny, nz}, t);
    }
    if (!rc && lineno == 0) {
        set_error("edt_tuning_cache_load: %s is empty", path);
        rc = EDT_ERR_ARG;
    }
    std::fclose(f);
    if (rc) return rc;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    for (const auto& e : got) g_tuned[e.first] = e.second;
    return (int)got.size();
}

int edt_tuning_cache_clear(void)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tuned.clear();
    return EDT_OK;
}

}  // extern "C"
