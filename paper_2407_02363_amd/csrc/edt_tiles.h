#pragma once
// Device code of the exact squared EDT tiles, shared by the per-map kernels
// (edt_core.hip) and the persistent batched kernel (batch.hip).
//
// The transform is separable (Sec. III-C, Alg. 1).  Step 1 finds the nearest
// site within each row; step 2 keeps, per column, the proximate sites (those
// whose distance function reaches the lower envelope of all of them); step 3
// reads every position of the column off that envelope; step 4 repeats
// steps 2-3 along z over the 2D results.  Every step keeps the smaller
// coordinate on equal distance, so with the passes in x, y, z order the site
// is the smallest linear index among the equidistant occupied voxels.
//
// Envelope arithmetic.  A site at position p with accumulated squared
// distance h contributes f(q) = h + (q - p)^2 = K - 2qp + q^2, K = h + p^2.
// The middle one of three sites a < b < c is dominated -- owns no stretch of
// the line -- iff (K_c - K_b)(b - a) <= (K_b - K_a)(c - b); a query moves to
// the next proximate site only while that one is strictly closer.
//
// Banding (the m2 / m3 bands of the paper's steps 2 and 3).  Each column is
// cut into NB bands; one thread per (column, band) builds the band's own
// envelope with a stack.  The band envelopes of a column are then merged:
// the envelope of two neighbouring chains keeps a prefix of the left one and
// a suffix of the right one, found by popping dominated sites on either side
// of the seam until neither side pops.  One thread per group of up to 4
// bands stitches the group's bands in order (a short chain of dependent
// steps); the groups then merge in log2(NB / 4) rounds of independent pairs.
// Each (column, band) thread then locates the envelope site of its first
// position (walking from its own band's range, then a binary search) and
// marches through its positions with a strength-reduced test.  The stacks
// keep packed self-contained entries (position | x' << 10 [| y' << 20]), so a
// key is recomputed from an entry and no side table is needed.
//
//   row records  one wave per group of whole rows (rows of 256 voxels or
//             more): per 64-column word, the word and the nearest occupied
//             column left and right of it, from ballots over the row's
//             bytes, written into the d2 buffer as scratch.
//   xy tile   work-group = (z slice, TW consecutive columns).  Per row, the
//             tile's 64-bit word plus the nearest set bit left and right of
//             it: read from the row records, or (narrower rows, and the
//             persistent batched kernel) cut out of the slice staged in LDS
//             as a bit string from 16-byte loads.  The (column, band) threads
//             derive x' per row from those and feed their stacks.  Output:
//             the 2D site x' | y' << 16 of every voxel, written into the site
//             buffer (0xFFFFFFFF if the slice is empty).
//   z tile    work-group = (row y, TW consecutive columns), all z.  Threads
//             load their band of the packed 2D sites (coalesced along x),
//             build, merge, query and overwrite d2 and site in place: every
//             read of a column happens before the first barrier and every
//             write after the last, and a column belongs to one work-group.
#include "common.h"


namespace edtmi {
namespace tiles {

constexpr int NT = 256;                 // threads per work-group
constexpr uint32_t XY_NONE = 0xFFFFFFFFu;
constexpr uint32_t POS_MASK = 1023u;

// 24-bit multiply (full rate on CDNA; v_mul_lo_u32 is quarter rate): exact
// when both operands fit in 24 signed bits and the product in 32.
__device__ __forceinline__ int mul24(int a, int b) { return __mul24(a, b); }

// Keys are below 3 * 1023^2 < 2^22 and position gaps below 2^10, so every
// operand fits in 24 bits; with all axes <= 512 the products stay below 2^31.
template <bool WIDE>
__device__ __forceinline__ bool dominated(int pa, int ka, int pb, int kb, int pc, int kc)
{
    if constexpr (WIDE) {
        return (int64_t)(kc - kb) * (pb - pa) <= (int64_t)(kb - ka) * (pc - pb);
    } else {
        return mul24(kc - kb, pb - pa) <= mul24(kb - ka, pc - pb);
    }
}

// f_1(q) < f_0(q); both sides carry the same q^2, and every term stays below
// 2^31 for positions and keys of grids up to 1024 per axis.
__device__ __forceinline__ bool next_closer(int p0, int k0, int p1, int k1, int q)
{
    return k1 - 2 * mul24(q, p1) < k0 - 2 * mul24(q, p0);
}

// entry of the y pass: y' | x' << 10
struct KeyY {
    int xc;
    __device__ __forceinline__ int operator()(uint32_t e) const
    {
        const int p = (int)(e & POS_MASK);
        const int d = xc - (int)(e >> 10);
        return mul24(d, d) + mul24(p, p);
    }
};

// entry of the z pass: z' | x' << 10 | y' << 20
struct KeyZ {
    int xc, yc;
    __device__ __forceinline__ int operator()(uint32_t e) const
    {
        const int p = (int)(e & POS_MASK);
        const int dx = xc - (int)((e >> 10) & POS_MASK);
        const int dy = yc - (int)(e >> 20);
        return mul24(dx, dx) + mul24(dy, dy) + mul24(p, p);
    }
};

// Band of this thread.  With tiles of 64 columns or more a wave is one band,
// and saying so lets the compiler keep band-wide positions and addresses in
// scalar registers.
template <int TW>
__device__ __forceinline__ int band_of()
{
    const int b = (int)threadIdx.x / TW;
    if constexpr (TW % 64 == 0) return __builtin_amdgcn_readfirstlane(b);
    return b;
}

// Band-local envelope of sites pushed in increasing position; the two
// topmost entries stay in registers.
template <int TW, bool WIDE, class KeyF>
struct BandStack {
    uint32_t* slot;   // this thread's slots, stride TW
    int top;
    int pa, ka, pb, kb;

    __device__ __forceinline__ void push(uint32_t e, int p, int k, const KeyF& key)
    {
        while (top >= 2 && dominated<WIDE>(pa, ka, pb, kb, p, k)) {
            --top;
            pb = pa;
            kb = ka;
            // the new second entry; with fewer than two left the value is
            // read from slot 0 and never used (one branch less per pop)
            const uint32_t ea = slot[(top >= 2 ? top - 2 : 0) * TW];
            pa = (int)(ea & POS_MASK);
            ka = key(ea);
        }
        slot[top * TW] = e;
        ++top;
        pa = pb;
        ka = kb;
        pb = p;
        kb = k;
    }
};

// Per-column band bookkeeping in LDS, [NB][TW] each: the surviving range
// [lo, hi) of every band's stack and the next band with a non-empty range.
struct BandMeta {
    int16_t* lo;
    int16_t* hi;
    int16_t* nxt;     // next band with a non-empty range (NB if none)
    int16_t* prv;     // previous band with a non-empty range (-1 if none)
};

// Merge the envelope of bands [gl, gm) (already merged) with that of bands
// [gm, gr): the result keeps a prefix of the left chain and a suffix of the
// right one, found by popping the seam's dominated sites on either side
// until neither side pops.  s, t are the left chain's last two sites, c, d
// the right chain's first two; all four stay in registers.  Only this
// thread touches bands [gl, gr) meanwhile.
template <int TW, bool WIDE, class KeyF>
__device__ void merge_group(const uint32_t* ent, int L, int col, const BandMeta& m, const KeyF& key,
                            int gl, int gm, int gr)
{
    auto E = [&](int b, int i) { return ent[(mul24(b, L) + i) * TW + col]; };
    auto LO = [&](int b) -> int16_t& { return m.lo[b * TW + col]; };
    auto HI = [&](int b) -> int16_t& { return m.hi[b * TW + col]; };
    int lastL = gm - 1;
    while (lastL >= gl && LO(lastL) == HI(lastL)) --lastL;
    if (lastL < gl) return;
    int firstR = gm;
    while (firstR < gr && LO(firstR) == HI(firstR)) ++firstR;
    if (firstR >= gr) return;
    int cntL = 0, cntR = 0;
    for (int b = gl; b < gm; ++b) cntL += HI(b) - LO(b);
    for (int b = gm; b < gr; ++b) cntR += HI(b) - LO(b);
    int loL = LO(lastL), hiL = HI(lastL), loR = LO(firstR), hiR = HI(firstR);
    // neighbouring non-empty bands inside the group (they exist when asked)
    auto prevL = [&](int b) {
        int p = b - 1;
        while (p > gl && LO(p) == HI(p)) --p;
        return p;
    };
    auto nextR = [&](int b) {
        int x = b + 1;
        while (x < gr - 1 && LO(x) == HI(x)) ++x;
        return x;
    };
    auto secondL = [&]() {
        if (hiL - loL >= 2) return E(lastL, hiL - 2);
        const int p = prevL(lastL);
        return E(p, HI(p) - 1);
    };
    auto secondR = [&]() {
        if (hiR - loR >= 2) return E(firstR, loR + 1);
        const int x = nextR(firstR);
        return E(x, LO(x));
    };
    uint32_t e = E(lastL, hiL - 1);
    int pt = (int)(e & POS_MASK), kt = key(e);
    int ps = 0, ks = 0;
    if (cntL >= 2) {
        e = secondL();
        ps = (int)(e & POS_MASK);
        ks = key(e);
    }
    e = E(firstR, loR);
    int pc = (int)(e & POS_MASK), kc = key(e);
    int pd = 0, kd = 0;
    if (cntR >= 2) {
        e = secondR();
        pd = (int)(e & POS_MASK);
        kd = key(e);
    }
    for (;;) {
        if (cntL >= 2 && dominated<WIDE>(ps, ks, pt, kt, pc, kc)) {
            --hiL;
            --cntL;
            if (hiL == loL) {
                HI(lastL) = (int16_t)hiL;
                lastL = prevL(lastL);
                loL = LO(lastL);
                hiL = HI(lastL);
            }
            pt = ps;
            kt = ks;
            if (cntL >= 2) {
                e = secondL();
                ps = (int)(e & POS_MASK);
                ks = key(e);
            }
            continue;
        }
        if (cntR >= 2 && dominated<WIDE>(pt, kt, pc, kc, pd, kd)) {
            ++loR;
            --cntR;
            if (loR == hiR) {
                LO(firstR) = (int16_t)loR;
                firstR = nextR(firstR);
                loR = LO(firstR);
                hiR = HI(firstR);
            }
            pc = pd;
            kc = kd;
            if (cntR >= 2) {
                e = secondR();
                pd = (int)(e & POS_MASK);
                kd = key(e);
            }
            continue;
        }
        break;
    }
    HI(lastL) = (int16_t)hiL;
    LO(firstR) = (int16_t)loR;
}

// Links between the non-empty band ranges of one column.
template <int TW, int NB>
__device__ void link_bands(int col, const BandMeta& m)
{
    int nxt = NB;
    for (int b = NB - 1; b >= 0; --b) {
        m.nxt[b * TW + col] = (int16_t)nxt;
        if (m.lo[b * TW + col] < m.hi[b * TW + col]) nxt = b;
    }
    int prv = -1;
    for (int b = 0; b < NB; ++b) {
        m.prv[b * TW + col] = (int16_t)prv;
        if (m.lo[b * TW + col] < m.hi[b * TW + col]) prv = b;
    }
}

// The envelope of bands [b0, b0 + G) of one column by one thread, left to
// right: the merged chain of bands [b0, r) takes band r by popping dominated
// sites on either side of the seam (the rule of merge_group; the envelope is
// unique, so the order of merging does not change it).  The chain's last two
// sites stay in registers; the range of every band finished with is written
// back.  After the build every band's range is [0, top).
template <int TW, int G, bool WIDE, class KeyF>
__device__ void stitch_bands(const uint32_t* ent, int L, int col, const BandMeta& m, const KeyF& key,
                             int b0)
{
    auto E = [&](int b, int i) { return ent[(mul24(b, L) + i) * TW + col]; };
    auto LO = [&](int b) -> int16_t& { return m.lo[b * TW + col]; };
    auto HI = [&](int b) -> int16_t& { return m.hi[b * TW + col]; };
    // last non-empty band before b (exists whenever the chain holds a site there)
    auto prev_band = [&](int b) {
        --b;
        while (b > b0 && LO(b) == HI(b)) --b;
        return b;
    };
    int top[G];
#pragma unroll
    for (int i = 0; i < G; ++i) top[i] = HI(b0 + i);
    int t = 0, lo_t = 0, hi_t = 0, cnt = 0;   // the chain's tail band, its range, chain length
    int p0 = 0, k0 = 0, p1 = 0, k1 = 0;       // the chain's second-to-last and last sites
#pragma unroll
    for (int i = 0; i < G; ++i) {
        const int r = b0 + i;
        const int n = top[i];
        if (n == 0) continue;
        const uint32_t ec = E(r, 0), ed = E(r, n > 1 ? 1 : 0);
        const uint32_t ey = E(r, n > 1 ? n - 2 : 0), ez = E(r, n - 1);
        if (cnt == 0) {
            t = r;
            lo_t = 0;
            hi_t = n;
            cnt = n;
            p1 = (int)(ez & POS_MASK);
            k1 = key(ez);
            p0 = (int)(ey & POS_MASK);
            k0 = key(ey);
            continue;
        }
        int lo_r = 0, rem = n;
        int pc = (int)(ec & POS_MASK), kc = key(ec);
        int pd = (int)(ed & POS_MASK), kd = key(ed);
        for (;;) {
            if (cnt >= 2 && dominated<WIDE>(p0, k0, p1, k1, pc, kc)) {
                --hi_t;
                --cnt;
                p1 = p0;
                k1 = k0;
                if (hi_t == lo_t) {
                    HI(t) = (int16_t)hi_t;
                    t = prev_band(t);
                    lo_t = LO(t);
                    hi_t = HI(t);
                }
                if (cnt >= 2) {
                    uint32_t e;
                    if (hi_t - lo_t >= 2) {
                        e = E(t, hi_t - 2);
                    } else {
                        const int b = prev_band(t);
                        e = E(b, HI(b) - 1);
                    }
                    p0 = (int)(e & POS_MASK);
                    k0 = key(e);
                }
                continue;
            }
            if (rem >= 2 && dominated<WIDE>(p1, k1, pc, kc, pd, kd)) {
                ++lo_r;
                --rem;
                pc = pd;
                kc = kd;
                if (rem >= 2) {
                    const uint32_t e = E(r, lo_r + 1);
                    pd = (int)(e & POS_MASK);
                    kd = key(e);
                }
                continue;
            }
            break;
        }
        HI(t) = (int16_t)hi_t;
        LO(r) = (int16_t)lo_r;
        // band r becomes the chain's tail; its last two sites are untouched
        // unless a single one is left
        cnt += rem;
        if (rem >= 2) {
            p1 = (int)(ez & POS_MASK);
            k1 = key(ez);
            p0 = (int)(ey & POS_MASK);
            k0 = key(ey);
        } else {
            p0 = p1;
            k0 = k1;
            p1 = pc;
            k1 = kc;
        }
        t = r;
        lo_t = lo_r;
        hi_t = n;
    }
}

// All bands of every column of the tile, then the band links.  Groups of up
// to 4 bands are stitched in sequence, one thread per group; the groups then
// merge in log2(NB / 4) rounds of independent pairs, so the chain of
// dependent steps stays short for any band count.
template <int TW, int NB, bool WIDE, class KeyF>
__device__ __forceinline__ void merge_all(const uint32_t* ent, int L, int col, int band, bool live,
                                          const BandMeta& m, const KeyF& key)
{
    if constexpr (NB <= 4) {
        if (live && band == col * NB / TW) {
            stitch_bands<TW, NB, WIDE>(ent, L, col, m, key, 0);
            link_bands<TW, NB>(col, m);
        }
    } else {
        if (live && (band & 3) == 0) stitch_bands<TW, 4, WIDE>(ent, L, col, m, key, band);
        __syncthreads();
        for (int half = 4; half < NB; half <<= 1) {
            const int span = half << 1;
            if (live && (band & (span - 1)) == 0)
                merge_group<TW, WIDE>(ent, L, col, m, key, band, band + half, band + span);
            __syncthreads();
        }
        if (live && band == col * NB / TW) link_bands<TW, NB>(col, m);
    }
    __syncthreads();
}

// Positions [q0, q1) of one column off the merged envelope.  The site of
// q0 is found first (scan over band ranges, binary search inside one); then
// the march moves to the next envelope site while it is strictly closer:
// with dK = K1 - K0 and dp2 = 2 (p1 - p0) > 0 that is dK < q * dp2, kept as
// a running difference.  begin(q, entry, pos, key) is called whenever the
// site changes (and at q0), step(q) once per position; none(q0, q1) if the
// column has no site.
template <int TW, int NB, class KeyF, class Begin, class Step, class None>
__device__ __forceinline__ void query_band(const uint32_t* ent, int L, int col, const BandMeta& m,
                                           int q0, int q1, const KeyF& key, Begin begin, Step step,
                                           None none)
{
    auto E = [&](int b, int i) { return ent[(mul24(b, L) + i) * TW + col]; };
    auto LO = [&](int b) -> int { return m.lo[b * TW + col]; };
    auto HI = [&](int b) -> int { return m.hi[b * TW + col]; };
    auto NX = [&](int b) -> int { return m.nxt[b * TW + col]; };
    auto PV = [&](int b) -> int { return m.prv[b * TW + col]; };
    // start from the nearest non-empty band to this one and walk to the band
    // range holding the envelope site of q0
    const int own = q0 / L;
    int j;
    if (LO(own) < HI(own)) j = own;
    else if (NX(own) < NB) j = NX(own);
    else if (PV(own) >= 0) j = PV(own);
    else {
        none(q0, q1);
        return;
    }
    int k;
    for (;;) {
        const int hij = HI(j);
        const int jn = NX(j);
        if (jn < NB) {
            const uint32_t el = E(j, hij - 1), en = E(jn, LO(jn));
            if (next_closer((int)(el & POS_MASK), key(el), (int)(en & POS_MASK), key(en), q0)) {
                j = jn;
                continue;
            }
        }
        const int jp = PV(j);
        if (jp >= 0) {
            const uint32_t el = E(jp, HI(jp) - 1), ef = E(j, LO(j));
            if (!next_closer((int)(el & POS_MASK), key(el), (int)(ef & POS_MASK), key(ef), q0)) {
                j = jp;
                continue;
            }
        }
        int a = LO(j), b = hij - 1;
        while (a < b) {
            const int mid = (a + b) >> 1;
            const uint32_t e0 = E(j, mid), e1 = E(j, mid + 1);
            if (next_closer((int)(e0 & POS_MASK), key(e0), (int)(e1 & POS_MASK), key(e1), q0))
                a = mid + 1;
            else
                b = mid;
        }
        k = a;
        break;
    }
    uint32_t ek = E(j, k);
    int pk = (int)(ek & POS_MASK), kk = key(ek);
    // the current band's end and where the envelope goes on after it, kept
    // in registers and refreshed only when the march changes band
    int hij = HI(j), jnx = NX(j);
    int lonx = jnx < NB ? LO(jnx) : 0;
    // next site and the running test value g(q) = q * dp2 - dK (advance iff g > 0)
    int jn = 0, kn = 0, pn = 0, kkn = 0, dp2 = 0, g = 0;
    uint32_t en = 0;
    bool has_next = false;
    auto load_next = [&](int q) {
        const bool same = k + 1 < hij;
        jn = same ? j : jnx;
        kn = same ? k + 1 : lonx;
        has_next = jn < NB;
        // past the column's last site, read the current one (value unused)
        en = E(has_next ? jn : j, has_next ? kn : k);
        pn = (int)(en & POS_MASK);
        kkn = key(en);
        dp2 = 2 * (pn - pk);
        g = mul24(q, dp2) - (kkn - kk);
    };
    load_next(q0);
    begin(q0, ek, pk, kk);
    for (int q = q0; q < q1; ++q) {
        if (has_next && g > 0) {
            do {
                if (jn != j) {
                    hij = HI(jn);
                    jnx = NX(jn);
                    lonx = jnx < NB ? LO(jnx) : 0;
                }
                j = jn;
                k = kn;
                ek = en;
                pk = pn;
                kk = kkn;
                load_next(q);
            } while (has_next && g > 0);
            begin(q, ek, pk, kk);
        }
        step(q);
        g += dp2;
    }
}

// bit i set iff byte i of w is nonzero
__device__ __forceinline__ uint32_t nonzero_bytes(uint32_t w)
{
    uint32_t t = w | (w >> 4);
    t |= t >> 2;
    t |= t >> 1;
    t &= 0x01010101u;
    return (t * 0x01020408u) >> 24;
}

// ---------------------------------------------------------------------------
// steps 1-3 per (slice, column tile)
// ---------------------------------------------------------------------------
// Words of the 16-byte row path's staging buffer in LDS (8 KiB).
constexpr int XSTAGE_WORDS = 1024;

// Dynamic LDS of k_edt_xy: envelope entries (or the row staging buffer,
// whichever is larger) plus three row-record arrays.
__host__ __device__ inline size_t z_lds(int tw, int nzv, int nt = NT)
{
    return (size_t)4 * nt * ((nzv + nt / tw - 1) / (nt / tw));
}

__host__ __device__ inline size_t xy_lds(int tw, int nyv, int nt = NT)
{
    const size_t ent = (size_t)4 * nt * ((nyv + nt / tw - 1) / (nt / tw));
    return (ent > 8 * (size_t)XSTAGE_WORDS ? ent : 8 * (size_t)XSTAGE_WORDS) + 12 * (size_t)nyv;
}

// One xy tile: slice z, columns [x0, x0 + TW), T = z * ntx + x0 / TW.
// Steps 2-3 of one xy tile from its row records: per row y of slice z, the
// tile's 64-bit occupancy word rword[y] (columns [64 w0, 64 w0 + 64)) and the
// nearest occupied column left (rleft) and right (rright) of that word, -1
// if none.  Writes the 2D site of every voxel of the tile.
template <int TW, bool WIDE, int NTX>
__device__ __forceinline__ void xy_bands(uint32_t* ent, const uint64_t* rword, const int16_t* rleft,
                                         const int16_t* rright, uint32_t* __restrict__ xy, int nx,
                                         int ny, int z, int x0, int w0, int L)
{
    constexpr int NB = NTX / TW;
    __shared__ int16_t s_lo[NB * TW], s_hi[NB * TW], s_nxt[NB * TW], s_prv[NB * TW];
    const BandMeta meta{s_lo, s_hi, s_nxt, s_prv};

    // ---- step 2, band-local: x' per row from the row records, then push
    const int col = threadIdx.x % TW;
    const int band = band_of<TW>();
    const int xc = x0 + col;
    const bool live = xc < nx;
    const KeyY key{xc};
    const int q0 = band * L;
    const int q1 = min(ny, q0 + L);
    {
        const int bit = (x0 & 63) + col;
        const uint64_t lmask = (2ull << bit) - 1ull;
        const uint64_t rmask = ~0ull << bit;
        BandStack<TW, WIDE, KeyY> st{ent + q0 * TW + col, 0, 0, 0, 0, 0};
        if (live) {
            for (int y = q0; y < q1; ++y) {
                const uint64_t mk = rword[y];
                const uint64_t lm = mk & lmask, rm = mk & rmask;
                const int xl = lm ? (w0 * 64 + 63 - __clzll(lm)) : (int)rleft[y];
                const int xr = rm ? (w0 * 64 + __ffsll((unsigned long long)rm) - 1) : (int)rright[y];
                int xp;
                if (xl < 0) xp = xr;
                else if (xr < 0) xp = xl;
                else xp = (xc - xl <= xr - xc) ? xl : xr;
                if (xp < 0) continue;
                const int d = xc - xp;
                st.push((uint32_t)y | ((uint32_t)xp << 10), y, mul24(d, d) + mul24(y, y), key);
            }
        }
        s_lo[band * TW + col] = 0;
        s_hi[band * TW + col] = (int16_t)st.top;
    }
    __syncthreads();
    merge_all<TW, NB, WIDE>(ent, L, col, band, live, meta, key);

    // ---- step 3: every row of the band
    if (!live || q0 >= q1) return;
    // band-wide row pointer (scalar when a wave is one band); the lane adds its column
    uint32_t* row = xy + ((size_t)z * ny + q0) * nx + x0;
    uint32_t val = 0;
    query_band<TW, NB>(
        ent, L, col, meta, q0, q1, key,
        [&](int, uint32_t e, int, int) { val = (e >> 10) | ((e & POS_MASK) << 16); },
        [&](int) {
            row[col] = val;
            row += nx;
        },
        [&](int a, int b) {
            for (int q = a; q < b; ++q, row += nx) row[col] = XY_NONE;
        });}

template <int TW, bool WIDE, int NTX = NT>
__device__ __forceinline__ void edt_xy_tile(const uint8_t* __restrict__ occ,
                                            uint32_t* __restrict__ xy, int nx, int ny, int nz,
                                            int ntx, int T, uint32_t* lds)
{
    constexpr int NB = NTX / TW;
    constexpr int XCH = 8;   // 16-byte loads in flight per thread
    const int L = (ny + NB - 1) / NB;
    // step 1 stages rows in the envelope area, which is only written after it
    const int ent_words = max(NB * L * TW, 2 * XSTAGE_WORDS);
    uint32_t* ent = lds;                                                // [NB*L][TW]
    uint64_t* stage = reinterpret_cast<uint64_t*>(lds);                 // [XSTAGE_WORDS]
    uint64_t* rword = reinterpret_cast<uint64_t*>(lds + ent_words);     // [ny]
    int16_t* rleft = reinterpret_cast<int16_t*>(rword + ny);            // [ny]
    int16_t* rright = rleft + ny;                                       // [ny]
    const int z = T / ntx;
    const int x0 = (T - z * ntx) * TW;
    const int w0 = x0 >> 6;
    const int nwords = (nx + 63) >> 6;

    // ---- step 1: per row, the tile's 64-bit occupancy word and the nearest
    // occupied voxel left and right of the word.  Blocks of whole rows arrive
    // as 16-byte loads from 16-byte aligned addresses and become 16-bit masks
    // in LDS (bit b of the block = byte b - off of the block's first row);
    // one thread per row then cuts its row's 64-column words out of the bit
    // string.  Only a chunk that sticks out of the buffer (the first one when
    // occ is not 16-byte aligned, the last one when the end is not) is read
    // byte by byte, so no load leaves [occ, occ + n).
    {
        constexpr int SBITS = XSTAGE_WORDS * 64;
        const long long n = (long long)nx * ny * nz;
        const int mis = (int)((uintptr_t)occ & 15u);
        const uint4* base16 = reinterpret_cast<const uint4*>(occ - mis);
        // chunk k covers bytes [16k - mis, 16k - mis + 16) of occ; the whole
        // ones are k in [kf, ke)
        const long long kf = mis ? 1 : 0;
        const long long ke = (n + mis) >> 4;
        const bool any_whole = ke > kf;
        const int rblk = min(ny, (SBITS - 32) / nx);
        uint16_t* stage16 = reinterpret_cast<uint16_t*>(stage);
        for (int y0 = 0; y0 < ny; y0 += rblk) {
            const int rows = min(rblk, ny - y0);
            const long long fs = ((long long)z * ny + y0) * nx;
            const long long c0 = (fs + mis) >> 4;
            const int off = (int)((fs + mis) & 15);
            const int nch = (int)(((fs + (long long)rows * nx - 1 + mis) >> 4) - c0 + 1);
            for (int i0 = 0; i0 < nch; i0 += NTX * XCH) {
                uint4 v[XCH];
                if (any_whole) {
#pragma unroll
                    for (int u = 0; u < XCH; ++u) {
                        long long k = c0 + min(i0 + u * NTX + (int)threadIdx.x, nch - 1);
                        k = k < kf ? kf : (k >= ke ? ke - 1 : k);
                        v[u] = base16[k];
                    }
                }
#pragma unroll
                for (int u = 0; u < XCH; ++u) {
                    const int i = i0 + u * NTX + (int)threadIdx.x;
                    if (i < nch) {
                        const long long k = c0 + i;
                        uint32_t m = 0;
                        if (k >= kf && k < ke) {
                            m = nonzero_bytes(v[u].x) | (nonzero_bytes(v[u].y) << 4) |
                                (nonzero_bytes(v[u].z) << 8) | (nonzero_bytes(v[u].w) << 12);
                        } else {
                            for (int j = 0; j < 16; ++j) {
                                const long long f = 16 * k + j - mis;
                                if (f >= 0 && f < n && occ[f]) m |= 1u << j;
                            }
                        }
                        stage16[i] = (uint16_t)m;
                    }
                }
            }
            __syncthreads();
            for (int r = threadIdx.x; r < rows; r += NTX) {
                const int rb = off + r * nx;
                // columns [64c, 64c + 64) of row r, bits past the row end cleared
                auto word = [&](int c) -> uint64_t {
                    const int b = rb + 64 * c;
                    const int wi = b >> 6, sh = b & 63;
                    uint64_t w = stage[wi] >> sh;
                    if (sh) w |= stage[min(wi + 1, XSTAGE_WORDS - 1)] << (64 - sh);
                    const int valid = nx - 64 * c;
                    return valid >= 64 ? w : (w & ((1ull << valid) - 1ull));
                };
                int left = -1, right = -1;
                for (int c = w0 - 1; c >= 0; --c) {
                    const uint64_t w = word(c);
                    if (w) {
                        left = c * 64 + 63 - __clzll(w);
                        break;
                    }
                }
                for (int c = w0 + 1; c < nwords; ++c) {
                    const uint64_t w = word(c);
                    if (w) {
                        right = c * 64 + __ffsll((unsigned long long)w) - 1;
                        break;
                    }
                }
                rword[y0 + r] = word(w0);
                rleft[y0 + r] = (int16_t)left;
                rright[y0 + r] = (int16_t)right;
            }
            __syncthreads();
        }
    }

    xy_bands<TW, WIDE, NTX>(ent, rword, rleft, rright, xy, nx, ny, z, x0, w0, L);
}

// ---------------------------------------------------------------------------
// step 1 once per row, then steps 2-3 per (slice, column tile)
// ---------------------------------------------------------------------------
// Row records of a whole map, for rows of at least 64 voxels: per row (z, y)
// and 64-column word w, the word (bit i = column 64 w + i occupied) and the
// nearest occupied column left and right of it (-1 if none).  They live in
// the d2 buffer, which the xy pass does not use and the z pass overwrites:
// 12 bytes per word against 4 * 64 bytes of d2 per word, from the first
// 8-byte boundary of d2 on.
struct RowRecords {
    uint64_t* word;
    int16_t* left;
    int16_t* right;
};

__host__ __device__ inline RowRecords row_records(int32_t* d2, int nx, int ny, int nz)
{
    const size_t rows = (size_t)ny * nz;
    const size_t nw = (size_t)((nx + 63) >> 6);
    const uintptr_t base = ((uintptr_t)d2 + 7) & ~(uintptr_t)7;
    RowRecords r;
    r.word = reinterpret_cast<uint64_t*>(base);
    r.left = reinterpret_cast<int16_t*>(r.word + rows * nw);
    r.right = r.left + rows * nw;
    return r;
}

// Rows read 4 bytes per lane: rows of a multiple of 4 bytes from a 4-byte
// aligned occupancy buffer.
__host__ __device__ inline bool record_words(const void* occ, int nx)
{
    return ((uintptr_t)occ & 3u) == 0 && (nx & 3) == 0;
}

// Rows per wave for the row records: whole rows, at most 16 loads per lane
// and (4 bytes per lane) 64 words per wave.
__host__ __device__ inline int record_rows_per_wave(const void* occ, int nx)
{
    const int nw = (nx + 63) >> 6, nch = (nx + 255) >> 8;
    if (!record_words(occ, nx)) return 16 / nw;
    const int a = 64 / nw, b = 16 / nch;
    return a < b ? a : b;
}

// Bits 0-15 of x spread to bits 0, 4, 8, ..., 60.
__device__ __forceinline__ uint64_t spread4(uint64_t x)
{
    x &= 0xFFFFull;
    x = (x | (x << 24)) & 0x000000FF000000FFull;
    x = (x | (x << 12)) & 0x000F000F000F000Full;
    x = (x | (x << 6)) & 0x0303030303030303ull;
    x = (x | (x << 3)) & 0x1111111111111111ull;
    return x;
}

// Every word's nearest occupied columns outside it within its row, for the
// words held by lanes [0, items), nw lanes per row, and the stores.
__device__ __forceinline__ void row_records_store(uint64_t mine, int items, int nw, size_t row0,
                                                  const RowRecords& rec)
{
    const int lane = (int)(threadIdx.x & 63);
    const uint64_t filled = __ballot(lane < items && mine != 0);
    const int rr = lane / nw;
    const int s0 = rr * nw, e0 = s0 + nw;          // the lanes of this lane's row
    const uint64_t lanes_below = ((1ull << lane) - 1ull) & ~((1ull << s0) - 1ull);
    const uint64_t lanes_above =
        (lane < 63 ? ~0ull << (lane + 1) : 0ull) & (e0 < 64 ? (1ull << e0) - 1ull : ~0ull);
    const uint64_t below = filled & lanes_below;
    const uint64_t above = filled & lanes_above;
    const int pw = below ? 63 - __clzll(below) : 0;
    const int qw = above ? __ffsll((unsigned long long)above) - 1 : 0;
    const uint64_t wl = __shfl(mine, pw);
    const uint64_t wr = __shfl(mine, qw);
    if (lane < items) {
        const size_t i = row0 * (size_t)nw + lane;
        rec.word[i] = mine;
        rec.left[i] = (int16_t)(below ? 64 * (pw - s0) + 63 - __clzll(wl) : -1);
        rec.right[i] = (int16_t)(above ? 64 * (qw - s0) + __ffsll((unsigned long long)wr) - 1 : -1);
    }
}

// The records of rows [row0, row0 + nrows), 4 bytes per lane: load j is the
// 256 bytes (four words) of chunk j % nch of row j / nch; one ballot per byte
// position gives, for each word of the chunk, every fourth bit.  Lane
// r * nw + w keeps the four ballots of its load and interleaves them into
// word w of row r.
__device__ __forceinline__ void row_summary_words(const uint8_t* __restrict__ occ, int nx, size_t row0,
                                                  int nrows, const RowRecords& rec)
{
    const int lane = (int)(threadIdx.x & 63);
    const int nw = (nx + 63) >> 6, nch = (nx + 255) >> 8;
    const int loads = nrows * nch;      // <= 16
    uint32_t v[16];
    {
        int rr = 0, k = 0;
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            const int x = 256 * k + 4 * lane;
            v[j] = (j < loads && x < nx)
                       ? *reinterpret_cast<const uint32_t*>(occ + (row0 + rr) * (size_t)nx + x)
                       : 0u;
            if (++k == nch) {
                k = 0;
                ++rr;
            }
        }
    }
    // lane r * nw + w holds word w of row r: load (r * nch + w / 4), quarter w % 4
    const int items = nrows * nw;
    const int wr_ = lane % nw;
    const int mine_load = lane < items ? (lane / nw) * nch + wr_ / 4 : -1;
    uint64_t a0 = 0, a1 = 0, a2 = 0, a3 = 0;
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        const uint64_t m0 = __ballot((v[j] & 0x000000FFu) != 0), m1 = __ballot((v[j] & 0x0000FF00u) != 0);
        const uint64_t m2 = __ballot((v[j] & 0x00FF0000u) != 0), m3 = __ballot((v[j] & 0xFF000000u) != 0);
        if (j == mine_load) {
            a0 = m0;
            a1 = m1;
            a2 = m2;
            a3 = m3;
        }
    }
    const int sh = 16 * (wr_ & 3);
    const uint64_t mine = spread4(a0 >> sh) | (spread4(a1 >> sh) << 1) | (spread4(a2 >> sh) << 2) |
                          (spread4(a3 >> sh) << 3);
    row_records_store(mine, items, nw, row0, rec);
}

// The records of rows [row0, row0 + nrows) of one map by one wave, nrows <=
// record_rows_per_wave(nx).  Item j (row j / nw, word j % nw) is the 64
// consecutive bytes one byte per lane; all loads are issued first, then one
// ballot per item gives its word, kept by lane j.  A ballot of the non-empty
// words and two shuffles give every word's nearest occupied columns outside
// it within its row.
__device__ __forceinline__ void row_summary(const uint8_t* __restrict__ occ, int nx, size_t row0,
                                            int nrows, const RowRecords& rec)
{
    const int lane = (int)(threadIdx.x & 63);
    const int nw = (nx + 63) >> 6;      // 1..16
    const int items = nrows * nw;       // <= 16
    uint8_t b[16];
    {
        int rr = 0, c = 0;
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            const int x = 64 * c + lane;
            b[j] = (j < items && x < nx) ? occ[(row0 + rr) * (size_t)nx + x] : (uint8_t)0;
            if (++c == nw) {
                c = 0;
                ++rr;
            }
        }
    }
    uint64_t mine = 0;                  // lane j keeps item j's word
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        const uint64_t w = __ballot(b[j] != 0);
        if (lane == j) mine = w;
    }
    row_records_store(mine, items, nw, row0, rec);
}

// Dynamic LDS of the xy tile that reads row records: envelope entries plus
// the three row-record arrays.
__host__ __device__ inline size_t xy_rows_lds(int tw, int nyv, int nt = NT)
{
    return (size_t)4 * nt * ((nyv + nt / tw - 1) / (nt / tw)) + 12 * (size_t)nyv;
}

// One xy tile (slice z, columns [x0, x0 + TW)) from the map's row records.
template <int TW, bool WIDE, int NTX = NT>
__device__ __forceinline__ void edt_xy_tile_rows(const RowRecords& rec, uint32_t* __restrict__ xy,
                                                 int nx, int ny, int ntx, int T, uint32_t* lds)
{
    constexpr int NB = NTX / TW;
    const int L = (ny + NB - 1) / NB;
    uint32_t* ent = lds;                                                  // [NB*L][TW]
    uint64_t* rword = reinterpret_cast<uint64_t*>(lds + NB * L * TW);     // [ny]
    int16_t* rleft = reinterpret_cast<int16_t*>(rword + ny);              // [ny]
    int16_t* rright = rleft + ny;                                         // [ny]
    const int z = T / ntx;
    const int x0 = (T - z * ntx) * TW;
    const int w0 = x0 >> 6;
    const int nw = (nx + 63) >> 6;
    for (int y = threadIdx.x; y < ny; y += NTX) {
        const size_t i = ((size_t)z * ny + y) * nw + w0;
        rword[y] = rec.word[i];
        rleft[y] = rec.left[i];
        rright[y] = rec.right[i];
    }
    __syncthreads();
    xy_bands<TW, WIDE, NTX>(ent, rword, rleft, rright, xy, nx, ny, z, x0, w0, L);
}

// ---------------------------------------------------------------------------
// step 4 per (row, column tile)
// ---------------------------------------------------------------------------
// One z tile: row y, columns [x0, x0 + TW), all z; T = y * ntx + x0 / TW.
template <int TW, bool WIDE, int NTZ = NT>
__device__ __forceinline__ void edt_z_tile(int32_t* d2, int32_t* site, int nx, int ny, int nz,
                                           int ntx, int T, uint32_t* lds)
{
    constexpr int NB = NTZ / TW;
    constexpr int CH = 8;   // positions per software-pipelined chunk
    const int L = (nz + NB - 1) / NB;
    uint32_t* ent = lds;    // [NB*L][TW]
    __shared__ int16_t s_lo[NB * TW], s_hi[NB * TW], s_nxt[NB * TW], s_prv[NB * TW];
    const BandMeta meta{s_lo, s_hi, s_nxt, s_prv};

    const int y = T / ntx;
    const int x0 = (T - y * ntx) * TW;
    const int col = threadIdx.x % TW;
    const int band = band_of<TW>();
    const int xc = x0 + col;
    const bool live = xc < nx;
    const KeyZ key{xc, y};
    const size_t plane = (size_t)nx * ny;
    const unsigned plane32 = (unsigned)nx * (unsigned)ny;
    const size_t base = (size_t)y * nx + xc;
    const int q0 = band * L;
    const int q1 = min(nz, q0 + L);

    {
        BandStack<TW, WIDE, KeyZ> st{ent + q0 * TW + col, 0, 0, 0, 0, 0};
        if (live && q0 < q1) {
            // chunks of CH positions, software-pipelined: the next chunk's
            // loads (clamped into the band) are in flight while this chunk is
            // pushed, with the chunk loop fully unrolled
            // row pointers are band-wide (scalar when a wave is one band),
            // the lane adds its column
            const uint32_t* tile_in = reinterpret_cast<const uint32_t*>(site) + ((size_t)y * nx + x0);
            auto load = [&](uint32_t (&v)[CH], int zb) {
#pragma unroll
                for (int i = 0; i < CH; ++i)   // z * plane < 2^32 with z < 2^10, plane <= 2^20
                    v[i] = (tile_in + __umul24((unsigned)min(zb + i, q1 - 1), plane32))[col];
            };
            uint32_t cur[CH], nxt[CH];
            load(cur, q0);
            for (int zb = q0; zb < q1; zb += CH) {
                load(nxt, zb + CH);
#pragma unroll
                for (int i = 0; i < CH; ++i) {
                    const int zz = zb + i;
                    if (zz < q1 && cur[i] != XY_NONE) {
                        const int xp = (int)(cur[i] & 0xFFFFu), yp = (int)(cur[i] >> 16);
                        const int dx = xc - xp, dy = y - yp;
                        st.push((uint32_t)zz | ((uint32_t)xp << 10) | ((uint32_t)yp << 20), zz,
                                mul24(dx, dx) + mul24(dy, dy) + mul24(zz, zz), key);
                    }
                }
#pragma unroll
                for (int i = 0; i < CH; ++i) cur[i] = nxt[i];
            }
        }
        s_lo[band * TW + col] = 0;
        s_hi[band * TW + col] = (int16_t)st.top;
    }
    __syncthreads();
    merge_all<TW, NB, WIDE>(ent, L, col, band, live, meta, key);

    if (!live || q0 >= q1) return;
    int dd = 0, inc = 0;
    int32_t ss = 0;
    // band-wide row pointers (scalar when a wave is one band)
    int32_t* row_d2 = d2 + ((size_t)y * nx + x0) + (size_t)q0 * plane;
    int32_t* row_site = site + ((size_t)y * nx + x0) + (size_t)q0 * plane;
    query_band<TW, NB>(
        ent, L, col, meta, q0, q1, key,
        [&](int q, uint32_t e, int p, int k) {
            // along a run of one site, (q - p)^2 + h grows by 2(q - p) + 1
            dd = k - 2 * mul24(q, p) + mul24(q, q);
            inc = 2 * (q - p) + 1;
            // x' + nx (y' + ny z'): 24-bit operands, product below 2^31
            ss = (int32_t)(((e >> 10) & POS_MASK) +
                           __umul24((unsigned)nx, (e >> 20) + __umul24((unsigned)ny, (unsigned)p)));
        },
        [&](int) {
            row_d2[col] = dd;
            row_site[col] = ss;
            row_d2 += plane;
            row_site += plane;
            dd += inc;
            inc += 2;
        },
        [&](int a, int b) {
            for (int q = a; q < b; ++q) {
                d2[base + (size_t)q * plane] = 0x7FFFFFFF;
                site[base + (size_t)q * plane] = -1;
            }
        });
}

}  // namespace tiles
}  // namespace edtmi
