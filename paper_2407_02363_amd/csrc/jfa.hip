// Jump flooding: the approximate transform the paper compares the exact one
// with (Sec. IV, Table 2).  Seeds are the occupied voxels; for step k = S/2,
// S/4, ..., 1 (S the smallest power of two >= the largest axis) every voxel
// keeps, among the sites held by itself and the 26 voxels at offsets in
// {-k, 0, k}^3 inside the grid, the one closest to it (squared voxel
// distance, the smaller linear index on ties).  One thread per voxel and
// step, reading the previous step's buffer.  Sites travel packed as
// x | y << 10 | z << 20, whose order is the linear-index order, and become
// linear indices (with their d2) in a last pass.
#include <algorithm>
#include <climits>

#include "common.h"

namespace edtmi {
namespace {

__global__ void k_jfa_init(const uint8_t* __restrict__ occ, int nx, int ny, int64_t n,
                           int32_t* __restrict__ out)
{
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    const int x = (int)(v % nx);
    const int64_t r = v / nx;
    const int y = (int)(r % ny), z = (int)(r / ny);
    out[v] = occ[v] ? (x | (y << 10) | (z << 20)) : -1;
}

__global__ void k_jfa_step(const int32_t* __restrict__ in, int32_t* __restrict__ out, int nx, int ny,
                           int nz, int k)
{
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t n = (int64_t)nx * ny * nz;
    if (v >= n) return;
    const int x = (int)(v % nx);
    const int64_t r = v / nx;
    const int y = (int)(r % ny), z = (int)(r / ny);
    int32_t best = -1;
    int bd = 0;
#pragma unroll
    for (int oz = -1; oz <= 1; ++oz) {
        const int qz = z + oz * k;
        if (qz < 0 || qz >= nz) continue;
#pragma unroll
        for (int oy = -1; oy <= 1; ++oy) {
            const int qy = y + oy * k;
            if (qy < 0 || qy >= ny) continue;
            const int64_t row = ((int64_t)qz * ny + qy) * nx;
#pragma unroll
            for (int ox = -1; ox <= 1; ++ox) {
                const int qx = x + ox * k;
                if (qx < 0 || qx >= nx) continue;
                const int32_t s = in[row + qx];
                if (s < 0) continue;
                const int dx = (s & 1023) - x, dy = ((s >> 10) & 1023) - y, dz = (s >> 20) - z;
                const int d = dx * dx + dy * dy + dz * dz;
                if (best < 0 || d < bd || (d == bd && s < best)) {
                    best = s;
                    bd = d;
                }
            }
        }
    }
    out[v] = best;
}

// packed site -> linear index and its squared distance (in place)
__global__ void k_jfa_finish(int32_t* __restrict__ site, int32_t* __restrict__ d2, int nx, int ny,
                             int64_t n)
{
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    const int32_t s = site[v];
    if (s < 0) {
        site[v] = -1;
        d2[v] = INT_MAX;
        return;
    }
    const int x = (int)(v % nx);
    const int64_t r = v / nx;
    const int y = (int)(r % ny), z = (int)(r / ny);
    const int sx = s & 1023, sy = (s >> 10) & 1023, sz = s >> 20;
    d2[v] = (sx - x) * (sx - x) + (sy - y) * (sy - y) + (sz - z) * (sz - z);
    site[v] = (int32_t)(sx + (int64_t)nx * (sy + (int64_t)ny * sz));
}

}  // namespace
}  // namespace edtmi

using namespace edtmi;

extern "C" {

size_t edt_jfa_workspace_bytes(const edt_grid_t* grid)
{
    if (check_grid(grid)) return 0;
    return (size_t)grid_voxels(grid) * 4;
}

int edt_jfa(const edt_grid_t* grid, const uint8_t* occ, int32_t* d2, int32_t* site, void* ws,
            size_t ws_bytes, void* stream)
{
    int rc = check_grid(grid);
    if (rc) return rc;
    if (!occ || !d2 || !site || !ws) {
        set_error("edt_jfa: NULL occ, d2, site or workspace");
        return EDT_ERR_ARG;
    }
    if (ws_bytes < edt_jfa_workspace_bytes(grid)) {
        set_error("edt_jfa: workspace of %zu bytes is below %zu", ws_bytes, edt_jfa_workspace_bytes(grid));
        return EDT_ERR_WORKSPACE;
    }
    const int64_t n = grid_voxels(grid);
    int S = 1, L = 0;
    while (S < grid->nx || S < grid->ny || S < grid->nz) {
        S <<= 1;
        ++L;
    }
    // the last step must land in site: start there after an even number of steps
    int32_t* buf[2] = {site, static_cast<int32_t*>(ws)};
    if (L & 1) std::swap(buf[0], buf[1]);
    const hipStream_t st = as_stream(stream);
    const unsigned blocks = (unsigned)((n + 255) / 256);
    hipLaunchKernelGGL(k_jfa_init, dim3(blocks), dim3(256), 0, st, occ, grid->nx, grid->ny, n, buf[0]);
    if ((rc = check_launch("k_jfa_init"))) return rc;
    int cur = 0;
    for (int k = S / 2; k >= 1; k /= 2) {
        hipLaunchKernelGGL(k_jfa_step, dim3(blocks), dim3(256), 0, st, buf[cur], buf[cur ^ 1], grid->nx,
                           grid->ny, grid->nz, k);
        if ((rc = check_launch("k_jfa_step"))) return rc;
        cur ^= 1;
    }
    hipLaunchKernelGGL(k_jfa_finish, dim3(blocks), dim3(256), 0, st, site, d2, grid->nx, grid->ny, n);
    return check_launch("k_jfa_finish");
}

}  // extern "C"
