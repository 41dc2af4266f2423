#pragma once
// Lean EDT tiles for the common map shapes (z <= 128 slices for the z pass,
// y <= 256 rows for the xy pass, every axis <= 512): one wave per band, so
// the positions a wave visits are wave-uniform, and the band envelopes are
// kept as per-lane masks of alive positions rather than as stacks.
//
// The mathematics is that of edt_tiles.h (Sec. III-C, Alg. 1): the lower
// envelope of the parabolas f(q) = h + (q - p)^2, the middle one of three
// sites a < b < c dominated iff (K_c - K_b)(b - a) <= (K_b - K_a)(c - b) with
// K = h + p^2, queries moving to the next envelope site only while it is
// strictly closer, the smaller coordinate winning every tie.  The dominance
// test is unchanged when an affine function of p is added to every K, so a
// band may take its positions relative to its first one while keeping the
// absolute K.
//
//   z tile   row y, 64 columns, ceil(nz / 32) bands of 32 positions.  Each
//            band loads its 32 positions (all loads in flight at once), keeps
//            K of every position in LDS and the alive positions of its
//            envelope as a 32-bit mask; a pop finds the new second entry as
//            the highest alive bit below the top.  One thread per column
//            stitches the bands; each band then rewrites its alive positions
//            as dx | dy << 11 | succ << 22 (dx = x - x', dy = y - y', succ =
//            the next alive position), and the queries follow succ.
//   xy tile  slice z, 64 columns, 8 bands of 32 rows.  The tile stages the
//            slice's row records (step 1) and a mask of its non-empty rows;
//            a band's build visits only the non-empty rows, computing x' of
//            its column from the record.  The band envelopes merge in a
//            pairwise tree (4, 2, 1 seams per column), the merged chain is
//            moved together, and each band queries its own rows.
#include "edt_tiles.h"

namespace edtmi {
namespace lean {

using tiles::mul24;
using tiles::RowRecords;
using tiles::XY_NONE;

// Positions of a 128-position column as two 64-bit masks.
struct Mask128 {
    uint64_t lo, hi;
    // highest set position < p (p in [0, 128]), or -1
    __device__ __forceinline__ int prev(int p) const
    {
        const uint64_t mh = p > 64 ? hi & (p >= 128 ? ~0ull : ((1ull << (p - 64)) - 1ull)) : 0ull;
        if (mh) return 127 - __clzll(mh);
        const uint64_t ml = lo & (p >= 64 ? ~0ull : ((1ull << p) - 1ull));
        return ml ? 63 - __clzll(ml) : -1;
    }
    // lowest set position > p (p in [-1, 127]), or -1
    __device__ __forceinline__ int next(int p) const
    {
        const uint64_t ml = p < 63 ? lo & (~0ull << (p + 1)) : 0ull;
        if (ml) return __ffsll((unsigned long long)ml) - 1;
        const uint64_t mh = p < 63 ? hi : (p < 127 ? hi & (~0ull << (p - 63)) : 0ull);
        return mh ? 63 + __ffsll((unsigned long long)mh) : -1;
    }
    __device__ __forceinline__ void clear(int p)
    {
        if (p < 64) lo &= ~(1ull << p);
        else hi &= ~(1ull << (p - 64));
    }
};

// K of a linked z entry dx | dy << 11 | succ << 22 at position p
__device__ __forceinline__ int z_key(uint32_t e, int p)
{
    const int dx = ((int)(e << 21)) >> 21, dy = ((int)(e << 10)) >> 21;
    return mul24(dx, dx) + mul24(dy, dy) + mul24(p, p);
}

constexpr int Z_MAX = 128;   // slices a lean z tile holds
constexpr int XY_MAX = 256;  // rows a lean xy tile holds
constexpr int XY_NB = 8;     // bands of 32 rows of a lean xy tile

// The local memory of one z tile and of one xy tile (the caller declares
// them, so that one persistent work-group can hold either).
struct ZLds {
    uint32_t val[Z_MAX * 64];   // per position: K, then the linked entry
    uint32_t msk[4 * 64];       // per band: alive positions
};
template <typename Ent>
struct XyLdsT {
    Ent stk[XY_NB * 32 * 64];        // [band][slot][col]: one envelope entry
    uint64_t rw[XY_MAX];             // the tile's word of every row
    int16_t rl[XY_MAX], rr[XY_MAX];  // nearest occupied column left / right of it
    uint32_t rmask[XY_MAX / 32];     // non-empty rows
    int16_t s_lo[XY_NB * 64], s_hi[XY_NB * 64];
};
// Entries x' | y' << 16 for any map; y' | |x - x'| << 8 for maps of at most
// 256 columns, which halves the stacks and so doubles the work-groups that
// fit per CU.
using XyLds = XyLdsT<uint32_t>;
using XyLdsN = XyLdsT<uint16_t>;

// ---------------------------------------------------------------------------
// z pass (step 4): tile T = y * ntx + x0 / 64 of a map with nz <= 128, by the
// 64 * ceil(nz_max / 32) threads tid = 0, 1, ... of a work-group (nz_max the
// largest nz of the launch; bands past this map's nz, or every band when
// nz = 0, only take part in the three barriers).  Reads the packed 2D sites
// from site and overwrites d2 and site in place: every global read happens
// before the first barrier, every write after the last, and a column
// belongs to one tile.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void z_tile(int32_t* d2, int32_t* site, int nx, int ny, int nz, int ntx, int T,
                                       int tid, ZLds& L)
{
    uint32_t* val = L.val;
    uint32_t* msk = L.msk;
    const int y = T / ntx;
    const int x0 = (T - y * ntx) * 64;
    const int col = tid & 63;
    const int band = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int xc = x0 + col;
    const bool live = xc < nx;
    const int xl = live ? xc : nx - 1;
    const int q0 = band * 32;
    const int n = min(32, nz - q0);        // <= 0 for bands past this map's nz
    const unsigned plane = (unsigned)nx * (unsigned)ny;
    uint32_t* vcol = val + col;
    uint32_t* vb = vcol + q0 * 64;

    // ---- the band's positions, all loads in flight, then its envelope
    uint32_t xr[32];   // dx | dy << 11 of each position, for the links
    uint32_t m = 0;
    if (n > 0) {
        const uint32_t* tin = reinterpret_cast<const uint32_t*>(site) + ((size_t)y * nx + xl) +
                              (size_t)q0 * plane;
#pragma unroll
        for (int i = 0; i < 32; ++i) xr[i] = tin[(size_t)min(i, n - 1) * plane];
        // top of the envelope (pb, kb), and dp = pb - pa, dk = kb - ka for the
        // entry below it (dp = 0, dk = -1 when there is none: never dominated)
        int pb = 0, kb = 0, dp = 0, dk = -1;
        bool any = false;
#pragma unroll
        for (int i = 0; i < 32; ++i) {
            if (i < n) {
                const uint32_t v = xr[i];
                const int z = q0 + i;
                const int dx = xc - (int)(v & 0xFFFFu), dy = y - (int)(v >> 16);
                const int K = mul24(dx, dx) + mul24(dy, dy) + z * z;
                vb[i * 64] = (uint32_t)K;
                xr[i] = ((uint32_t)dx & 0x7FFu) | (((uint32_t)dy & 0x7FFu) << 11);
                // an empty slice is empty in every column: the test is wave-uniform
                if (__builtin_amdgcn_readfirstlane(v) != XY_NONE) {
                    if (!any) {
                        any = true;
                        pb = i;
                        kb = K;
                        dp = 0;
                        dk = -1;
                        m = 1u << i;
                    } else {
                        while (mul24(K - kb, dp) <= mul24(dk, i - pb)) {
                            m ^= 1u << pb;
                            pb -= dp;
                            kb -= dk;
                            const uint32_t below = m & ((1u << pb) - 1u);
                            const int ia = 31 - __clz(below);
                            const int ka = (int)vb[max(ia, 0) * 64];
                            dp = below ? pb - ia : 0;
                            dk = below ? kb - ka : -1;
                        }
                        m |= 1u << i;
                        dp = i - pb;
                        dk = K - kb;
                        pb = i;
                        kb = K;
                    }
                }
            }
        }
    }
    msk[band * 64 + col] = m;
    __syncthreads();

    // ---- one thread per column stitches the bands left to right
    const int nb = (nz + 31) >> 5;
    auto K = [&](int p) { return (int)vcol[p * 64]; };
    auto dom = [&](int pa, int ka, int pb_, int kb_, int pc, int kc) {
        return mul24(kc - kb_, pb_ - pa) <= mul24(kb_ - ka, pc - pb_);
    };
    if (band == 0 && nb > 1) {
        uint32_t w[4];
#pragma unroll
        for (int b = 0; b < 4; ++b) w[b] = b < nb ? msk[b * 64 + col] : 0u;
        Mask128 M{(uint64_t)w[0] | ((uint64_t)w[1] << 32), (uint64_t)w[2] | ((uint64_t)w[3] << 32)};
#pragma unroll
        for (int j = 1; j < 4; ++j) {
            if (j >= nb || w[j] == 0) continue;
            const int t0 = M.prev(j * 32);
            if (t0 < 0) continue;
            // left chain: its last two sites t, s; right chain (band j): c, d
            int t = t0, kt = K(t);
            int s = M.prev(t), ks = K(max(s, 0));
            uint32_t wj = w[j];
            int c = j * 32 + __ffs(wj) - 1, kc = K(c);
            uint32_t rest = wj & (wj - 1u);
            int d = rest ? j * 32 + __ffs(rest) - 1 : -1, kd = K(max(d, 0));
            for (;;) {
                if (s >= 0 && dom(s, ks, t, kt, c, kc)) {
                    M.clear(t);
                    t = s;
                    kt = ks;
                    s = M.prev(t);
                    ks = K(max(s, 0));
                    continue;
                }
                if (d >= 0 && dom(t, kt, c, kc, d, kd)) {
                    M.clear(c);
                    wj &= wj - 1u;
                    c = d;
                    kc = kd;
                    rest = wj & (wj - 1u);
                    d = rest ? j * 32 + __ffs(rest) - 1 : -1;
                    kd = K(max(d, 0));
                    continue;
                }
                break;
            }
        }
        msk[0 * 64 + col] = (uint32_t)M.lo;
        msk[1 * 64 + col] = (uint32_t)(M.lo >> 32);
        msk[2 * 64 + col] = (uint32_t)M.hi;
        msk[3 * 64 + col] = (uint32_t)(M.hi >> 32);
    }
    __syncthreads();

    uint32_t w[4];
#pragma unroll
    for (int b = 0; b < 4; ++b) w[b] = b < nb ? msk[b * 64 + col] : 0u;
    const Mask128 M{(uint64_t)w[0] | ((uint64_t)w[1] << 32), (uint64_t)w[2] | ((uint64_t)w[3] << 32)};
    // ---- links: every alive position of this band gets dx | dy << 11 | succ << 22
    // (succ = the next alive position, the position itself at the last one)
    if (n > 0) {
        const uint32_t mine = w[band];
        const int after = M.next(q0 + 31);
        int sc = after >= 0 ? after : -1;
#pragma unroll
        for (int i = 31; i >= 0; --i) {
            if (i < n) {
                const int p = q0 + i;
                vb[i * 64] = xr[i] | ((uint32_t)(sc >= 0 ? sc : p) << 22);
                sc = (mine >> i) & 1u ? p : sc;
            }
        }
    }
    __syncthreads();

    // ---- queries of positions [q0, q0 + n)
    if (n <= 0) return;
    int32_t* od = d2 + ((size_t)y * nx + x0) + (size_t)q0 * plane;
    int32_t* os = site + ((size_t)y * nx + x0) + (size_t)q0 * plane;
    if ((M.lo | M.hi) == 0) {   // no occupied voxel in any slice
        if (live)
            for (int i = 0; i < n; ++i, od += plane, os += plane) {
                od[col] = 0x7FFFFFFF;
                os[col] = -1;
            }
        return;
    }
    auto KL = [&](int p) { return z_key(vcol[p * 64], p); };
    // the envelope site of q0: from the last alive position <= q0 (else the
    // first alive one), back while the previous is at least as close, else
    // forward while the next is closer (f is unimodal along the envelope)
    int t = M.prev(q0 + 1);
    if (t < 0) t = M.next(-1);
    int kt = KL(t);
    {
        int s = M.prev(t);
        bool back = false;
        while (s >= 0) {
            const int ks = KL(s);
            if (ks - 2 * mul24(q0, s) > kt - 2 * mul24(q0, t)) break;
            t = s;
            kt = ks;
            s = M.prev(t);
            back = true;
        }
        if (!back) {
            int u = M.next(t);
            while (u >= 0) {
                const int ku = KL(u);
                if (ku - 2 * mul24(q0, u) >= kt - 2 * mul24(q0, t)) break;
                t = u;
                kt = ku;
                u = M.next(t);
            }
        }
    }
    // x' + nx (y' + ny z'): 24-bit operands, product below 2^31
    auto site_of = [&](uint32_t e, int p) {
        const int dx = ((int)(e << 21)) >> 21, dy = ((int)(e << 10)) >> 21;
        return (int)((unsigned)(xc - dx) +
                     __umul24((unsigned)nx, (unsigned)(y - dy) + __umul24((unsigned)ny, (unsigned)p)));
    };
    // march: along a run of one site d2 grows by inc = 2 (q - p) + 1; the
    // next site u is strictly closer iff g = q * 2 (u - t) - (K_u - K_t) > 0
    uint32_t vt = vcol[t * 64];
    int dd = kt - 2 * mul24(q0, t) + mul24(q0, q0);
    int inc = 2 * (q0 - t) + 1;
    int ss = site_of(vt, t);
    int u = (int)(vt >> 22);
    uint32_t vu = vcol[u * 64];
    int ku = z_key(vu, u);
    int dp2 = 2 * (u - t);
    int g = u > t ? mul24(q0, dp2) - (ku - kt) : -1;
    for (int i = 0; i < n; ++i) {
        const int q = q0 + i;
        while (g > 0) {
            t = u;
            kt = ku;
            vt = vu;
            dd = kt - 2 * mul24(q, t) + mul24(q, q);
            inc = 2 * (q - t) + 1;
            ss = site_of(vt, t);
            u = (int)(vt >> 22);
            vu = vcol[u * 64];
            ku = z_key(vu, u);
            dp2 = 2 * (u - t);
            g = u > t ? mul24(q, dp2) - (ku - kt) : -1;
        }
        if (live) {
            od[col] = dd;
            os[col] = ss;
        }
        od += plane;
        os += plane;
        dd += inc;
        inc += 2;
        g += dp2;
    }
}

// ---------------------------------------------------------------------------
// xy pass (steps 2-3): tile T = z * ntx + x0 / 64 of a map with ny <= 256,
// from the map's row records; 512 threads.  Writes the 2D site x' | y' << 16
// of every voxel of the tile (0xFFFFFFFF if the slice is empty).  Ent =
// uint16_t needs nx <= 256.
// ---------------------------------------------------------------------------
template <typename Ent>
__device__ __forceinline__ void xy_tile(const RowRecords& rec, uint32_t* __restrict__ out, int nx, int ny,
                                        int ntx, int T, XyLdsT<Ent>& L)
{
    constexpr bool NARROW = sizeof(Ent) == 2;
    Ent* stk = L.stk;
    uint64_t* rw = L.rw;
    int16_t* rl = L.rl;
    int16_t* rr = L.rr;
    uint32_t* rmask = L.rmask;
    int16_t* s_lo = L.s_lo;
    int16_t* s_hi = L.s_hi;
    const int z = T / ntx;
    const int tx = T - z * ntx;
    const int x0 = tx * 64;
    const int nw = (nx + 63) >> 6;
    const int col = threadIdx.x & 63;
    const int band = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int xc = x0 + col;
    const bool live = xc < nx;

    if (threadIdx.x < XY_MAX) {
        const int yy = threadIdx.x;
        bool ne = false;
        if (yy < ny) {
            const size_t i = ((size_t)z * ny + yy) * nw + tx;
            const uint64_t w = rec.word[i];
            const int16_t l = rec.left[i], r = rec.right[i];
            rw[yy] = w;
            rl[yy] = l;
            rr[yy] = r;
            ne = w != 0 || l >= 0 || r >= 0;
        }
        const uint64_t b = __ballot(ne);
        if ((threadIdx.x & 63) == 0) {
            rmask[2 * (yy >> 6)] = (uint32_t)b;
            rmask[2 * (yy >> 6) + 1] = (uint32_t)(b >> 32);
        }
    }
    __syncthreads();
    const int y0 = band * 32;
    const int y1 = min(ny, y0 + 32);
    uint32_t* orow = out + (size_t)z * ny * nx + x0;
    {
        uint32_t any = 0;
#pragma unroll
        for (int k = 0; k < XY_MAX / 32; ++k) any |= rmask[k];
        if (__builtin_amdgcn_readfirstlane(any) == 0) {   // empty slice
            if (live)
                for (int yy = y0; yy < y1; ++yy) orow[(size_t)yy * nx + col] = XY_NONE;
            return;
        }
    }
    const uint64_t lmask = col == 63 ? ~0ull : ((2ull << col) - 1ull);   // columns <= xc
    const uint64_t hmask = ~0ull << col;                                   // columns >= xc
    // an entry's row y', its K = (x - x')^2 + y'^2, and the entry of (x', y')
    auto pos = [&](uint32_t e) -> int { return NARROW ? (int)(e & 0xFFu) : (int)(e >> 16); };
    auto key = [&](uint32_t e) {
        const int d = NARROW ? (int)(e >> 8) : xc - (int)(e & 0xFFFFu), p = pos(e);
        return mul24(d, d) + mul24(p, p);
    };
    auto make = [&](int xp, int yy) -> Ent {
        return NARROW ? (Ent)((uint32_t)yy | ((uint32_t)abs(xc - xp) << 8))
                      : (Ent)((uint32_t)xp | ((uint32_t)yy << 16));
    };
    // the site word x' | y' << 16 of an entry.  A narrow entry keeps |x - x'|
    // only: x' lies left of x exactly when the nearest occupied column at or
    // left of x in row y' is at that distance (step 1 gives ties to the left)
    auto site_word = [&](uint32_t e) -> uint32_t {
        if (!NARROW) return e;
        const int yq = (int)(e & 0xFFu), a = (int)(e >> 8);
        int xs = xc;
        if (a) {
            const uint64_t lm = rw[yq] & lmask;
            const int xl = lm ? x0 + 63 - __clzll(lm) : rl[yq];
            xs = xl >= 0 && xl == xc - a ? xc - a : xc + a;   // xl = -1: none on the left
        }
        return (uint32_t)xs | ((uint32_t)yq << 16);
    };
    Ent* scol = stk + col;
    auto E = [&](int b, int i) -> uint32_t { return scol[(b * 32 + i) * 64]; };

    // ---- band envelope over the band's non-empty rows (wave-uniform loop)
    {
        Ent* st = scol + band * 32 * 64;
        int top = 0, pa = 0, ka = 0, pb = 0, kb = 0;
        uint32_t bits = __builtin_amdgcn_readfirstlane(rmask[band]);
        while (bits) {
            const int yy = y0 + __builtin_ctz(bits);
            bits &= bits - 1u;
            // step 1: the nearest occupied column of row yy, ties to the left
            const uint64_t w = rw[yy];
            const int l = rl[yy], r = rr[yy];
            const uint64_t lm = w & lmask, hm = w & hmask;
            const int xlft = lm ? x0 + 63 - __clzll(lm) : l;
            const int xrgt = hm ? x0 + __ffsll((unsigned long long)hm) - 1 : r;
            const int xp = xlft < 0 ? xrgt : (xrgt < 0 ? xlft : (xc - xlft <= xrgt - xc ? xlft : xrgt));
            const int d = xc - xp;
            const int Kc = mul24(d, d) + mul24(yy, yy);
            while (top >= 2 && mul24(Kc - kb, pb - pa) <= mul24(kb - ka, yy - pb)) {
                --top;
                pb = pa;
                kb = ka;
                const uint32_t e = st[max(top - 2, 0) * 64];
                pa = pos(e);
                ka = key(e);
            }
            st[top * 64] = make(xp, yy);
            ++top;
            pa = pb;
            ka = kb;
            pb = yy;
            kb = Kc;
        }
        s_lo[band * 64 + col] = 0;
        s_hi[band * 64 + col] = (int16_t)top;
    }
    __syncthreads();

    // ---- merge the band envelopes: rounds of independent pairs
    int16_t* LO = s_lo + col;
    int16_t* HI = s_hi + col;
    // groups [gl, gm) and [gm, gr), each one chain of band ranges; the merged
    // chain keeps a prefix of the left one and a suffix of the right one
    auto merge = [&](int gl, int gm, int gr) {
        int lastL = gm - 1;
        while (lastL >= gl && LO[lastL * 64] == HI[lastL * 64]) --lastL;
        if (lastL < gl) return;
        int firstR = gm;
        while (firstR < gr && LO[firstR * 64] == HI[firstR * 64]) ++firstR;
        if (firstR >= gr) return;
        int cntL = 0, cntR = 0;
        for (int b = gl; b < gm; ++b) cntL += HI[b * 64] - LO[b * 64];
        for (int b = gm; b < gr; ++b) cntR += HI[b * 64] - LO[b * 64];
        int loL = LO[lastL * 64], hiL = HI[lastL * 64];
        int loR = LO[firstR * 64], hiR = HI[firstR * 64];
        auto secondL = [&]() -> uint32_t {
            if (hiL - loL >= 2) return E(lastL, hiL - 2);
            int p = lastL - 1;
            while (p > gl && LO[p * 64] == HI[p * 64]) --p;
            return E(p, HI[p * 64] - 1);
        };
        auto secondR = [&]() -> uint32_t {
            if (hiR - loR >= 2) return E(firstR, loR + 1);
            int x = firstR + 1;
            while (x < gr - 1 && LO[x * 64] == HI[x * 64]) ++x;
            return E(x, LO[x * 64]);
        };
        uint32_t e = E(lastL, hiL - 1);
        int pt = pos(e), kt = key(e);
        int ps = 0, ks = 0;
        if (cntL >= 2) {
            e = secondL();
            ps = pos(e);
            ks = key(e);
        }
        e = E(firstR, loR);
        int pc = pos(e), kc = key(e);
        int pd = 0, kd = 0;
        if (cntR >= 2) {
            e = secondR();
            pd = pos(e);
            kd = key(e);
        }
        for (;;) {
            if (cntL >= 2 && mul24(kc - kt, pt - ps) <= mul24(kt - ks, pc - pt)) {
                --hiL;
                --cntL;
                if (hiL == loL) {
                    HI[lastL * 64] = (int16_t)hiL;
                    --lastL;
                    while (lastL > gl && LO[lastL * 64] == HI[lastL * 64]) --lastL;
                    loL = LO[lastL * 64];
                    hiL = HI[lastL * 64];
                }
                pt = ps;
                kt = ks;
                if (cntL >= 2) {
                    e = secondL();
                    ps = pos(e);
                    ks = key(e);
                }
                continue;
            }
            if (cntR >= 2 && mul24(kd - kc, pc - pt) <= mul24(kc - kt, pd - pc)) {
                ++loR;
                --cntR;
                if (loR == hiR) {
                    LO[firstR * 64] = (int16_t)loR;
                    ++firstR;
                    while (firstR < gr - 1 && LO[firstR * 64] == HI[firstR * 64]) ++firstR;
                    loR = LO[firstR * 64];
                    hiR = HI[firstR * 64];
                }
                pc = pd;
                kc = kd;
                if (cntR >= 2) {
                    e = secondR();
                    pd = pos(e);
                    kd = key(e);
                }
                continue;
            }
            break;
        }
        HI[lastL * 64] = (int16_t)hiL;
        LO[firstR * 64] = (int16_t)loR;
    };
    if (band & 1) merge(band - 1, band, band + 1);
    __syncthreads();
    if ((band & 3) == 2) merge(band - 2, band, band + 2);
    __syncthreads();
    if (band == 4) merge(0, 4, 8);
    __syncthreads();

    // ---- the merged chain made contiguous: band b's surviving entries move
    // to [cum[b], cum[b + 1]) of the column (all read before any is written),
    // so that the queries index the chain directly
    int lo[XY_NB], cum[XY_NB + 1];
    cum[0] = 0;
#pragma unroll
    for (int b = 0; b < XY_NB; ++b) {
        lo[b] = LO[b * 64];
        cum[b + 1] = cum[b] + HI[b * 64] - lo[b];
    }
    const int n = cum[XY_NB];
    {
        uint32_t ev[32];
        const int mlo = lo[band], mcnt = cum[band + 1] - cum[band];
#pragma unroll
        for (int i = 0; i < 32; ++i) ev[i] = i < mcnt ? E(band, mlo + i) : 0u;
        __syncthreads();
#pragma unroll
        for (int i = 0; i < 32; ++i)
            if (i < mcnt) scol[(cum[band] + i) * 64] = (Ent)ev[i];
        __syncthreads();
    }

    // ---- queries of rows [y0, y1)
    if (y0 >= y1) return;
    auto at = [&](int j) -> uint32_t { return scol[j * 64]; };
    // the envelope site of y0 by binary search (f is unimodal along the chain)
    int a = 0, bb = n - 1;
    while (a < bb) {
        const int mid = (a + bb) >> 1;
        const uint32_t e0 = at(mid), e1 = at(mid + 1);
        if (key(e1) - 2 * mul24(y0, pos(e1)) < key(e0) - 2 * mul24(y0, pos(e0))) a = mid + 1;
        else bb = mid;
    }
    int j = a;
    uint32_t et = at(j);
    int pt = pos(et), kt = key(et);
    uint32_t en = at(min(j + 1, n - 1));
    int pn = pos(en), kn = key(en);
    int dp2 = 2 * (pn - pt);
    int g = j + 1 < n ? mul24(y0, dp2) - (kn - kt) : -1;
    uint32_t* o = orow + (size_t)y0 * nx;
    uint32_t sw = site_word(et);
    for (int yy = y0; yy < y1; ++yy) {
        if (g > 0) {
            do {
                ++j;
                et = en;
                pt = pn;
                kt = kn;
                en = at(min(j + 1, n - 1));
                pn = pos(en);
                kn = key(en);
                dp2 = 2 * (pn - pt);
                g = j + 1 < n ? mul24(yy, dp2) - (kn - kt) : -1;
            } while (g > 0);
            sw = site_word(et);
        }
        if (live) o[col] = sw;
        o += nx;
        g += dp2;
    }
}

}  // namespace lean
}  // namespace edtmi
