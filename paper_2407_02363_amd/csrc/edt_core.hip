// The exact squared EDT on gfx950 for one map: the xy-tile kernel (steps 1-3
// of Sec. III-C in every slice) and the z-tile kernel (step 4), their
// launchers and the tile heuristics.  The tile code is in edt_tiles.h.
#include "edt_tiles.h"

namespace edtmi {

namespace {

using namespace tiles;

template <int TW, bool WIDE>
__global__ __launch_bounds__(NT) void k_edt_xy(const uint8_t* __restrict__ occ,
                                               uint32_t* __restrict__ xy, int nx, int ny, int nz,
                                               int ntx)
{
    extern __shared__ uint32_t lds[];
    edt_xy_tile<TW, WIDE>(occ, xy, nx, ny, nz, ntx, xcd_remap(blockIdx.x, nz * ntx), lds);
}

template <int TW, bool WIDE, int NTZ>
__global__ __launch_bounds__(NTZ) void k_edt_z(int32_t* d2, int32_t* site, int nx, int ny, int nz,
                                               int ntx)
{
    extern __shared__ uint32_t lds[];
    edt_z_tile<TW, WIDE, NTZ>(d2, site, nx, ny, nz, ntx, xcd_remap(blockIdx.x, ny * ntx), lds);
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

template <int TW, bool WIDE>
int launch_xy_w(const edt_grid_t* g, const uint8_t* occ, uint32_t* xy, hipStream_t st)
{
    static bool done = false;
    int rc = allow_lds(k_edt_xy<TW, WIDE>, done);
    if (rc) return rc;
    const int ntx = (g->nx + TW - 1) / TW;
    const size_t lds = xy_lds(TW, g->ny);
    hipLaunchKernelGGL((k_edt_xy<TW, WIDE>), dim3(g->nz * ntx), dim3(NT), lds, st, occ,
                       xy, g->nx, g->ny, g->nz, ntx);
    return check_launch("k_edt_xy");
}

template <int TW>
int launch_xy_tw(const edt_grid_t* g, const uint8_t* occ, uint32_t* xy, bool wide, hipStream_t st)
{
    return wide ? launch_xy_w<TW, true>(g, occ, xy, st) : launch_xy_w<TW, false>(g, occ, xy, st);
}

template <int TW, bool WIDE, int NTZ>
int launch_z_t(const edt_grid_t* g, int32_t* d2, int32_t* site, hipStream_t st)
{
    static bool done = false;
    int rc = allow_lds(k_edt_z<TW, WIDE, NTZ>, done);
    if (rc) return rc;
    const int ntx = (g->nx + TW - 1) / TW;
    const size_t lds = z_lds(TW, g->nz, NTZ);
    hipLaunchKernelGGL((k_edt_z<TW, WIDE, NTZ>), dim3(g->ny * ntx), dim3(NTZ), lds, st, d2, site,
                       g->nx, g->ny, g->nz, ntx);
    return check_launch("k_edt_z");
}

template <int TW, int NTZ>
int launch_z_tw(const edt_grid_t* g, int32_t* d2, int32_t* site, bool wide, hipStream_t st)
{
    return wide ? launch_z_t<TW, true, NTZ>(g, d2, site, st) : launch_z_t<TW, false, NTZ>(g, d2, site, st);
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
        return xy_lds(tw, g->ny) <= LDS_MAX;
    }
    if (tw != 8 && tw != 16 && tw != 32 && tw != 64) return false;
    if (nt != 64 && nt != 128 && nt != 256) return false;
    if (tw > nt) return false;
    return z_lds(tw, g->nz, nt) <= LDS_MAX;
}

EdtTuning default_tuning(const edt_grid_t* g)
{
    // measured on MI355X: 32-wide xy tiles up to 256 rows, 16-wide beyond;
    // z tiles keep about 32 positions per band
    EdtTuning t;
    t.xy_tw = g->ny <= 256 ? 32 : 16;
    t.z_tw = g->nz <= 128 ? 64 : (g->nz <= 256 ? 32 : 16);
    t.z_nt = 256;
    if (!tile_ok(1, t.xy_tw, g, 256)) t.xy_tw = 16;
    if (!tile_ok(2, t.z_tw, g, t.z_nt)) t.z_tw = 8;
    return t;
}

int launch_edt_xy(const edt_grid_t* g, const uint8_t* occ, uint32_t* xy, int tw, hipStream_t st)
{
    const bool wide = needs_wide(g);
    switch (tw) {
        case 64: return launch_xy_tw<64>(g, occ, xy, wide, st);
        case 32: return launch_xy_tw<32>(g, occ, xy, wide, st);
        case 16: return launch_xy_tw<16>(g, occ, xy, wide, st);
        default: set_error("bad xy tile width %d", tw); return EDT_ERR_ARG;
    }
}

int launch_edt_z(const edt_grid_t* g, int32_t* d2, int32_t* site, int tw, int nt, hipStream_t st)
{
    const bool wide = needs_wide(g);
    if (nt == 256) {
        switch (tw) {
            case 64: return launch_z_tw<64, 256>(g, d2, site, wide, st);
            case 32: return launch_z_tw<32, 256>(g, d2, site, wide, st);
            case 16: return launch_z_tw<16, 256>(g, d2, site, wide, st);
            case 8: return launch_z_tw<8, 256>(g, d2, site, wide, st);
        }
    } else if (nt == 128) {
        switch (tw) {
            case 64: return launch_z_tw<64, 128>(g, d2, site, wide, st);
            case 32: return launch_z_tw<32, 128>(g, d2, site, wide, st);
            case 16: return launch_z_tw<16, 128>(g, d2, site, wide, st);
            case 8: return launch_z_tw<8, 128>(g, d2, site, wide, st);
        }
    } else if (nt == 64) {
        switch (tw) {
            case 64: return launch_z_tw<64, 64>(g, d2, site, wide, st);
            case 32: return launch_z_tw<32, 64>(g, d2, site, wide, st);
            case 16: return launch_z_tw<16, 64>(g, d2, site, wide, st);
            case 8: return launch_z_tw<8, 64>(g, d2, site, wide, st);
        }
    }
    set_error("bad z tile %d / group %d", tw, nt);
    return EDT_ERR_ARG;
}

}  // namespace edtmi
