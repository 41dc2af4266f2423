/*
 * CPU oracle for the distance-map hot path.  TEST INFRASTRUCTURE ONLY: the
 * tests, the smoke check and the benchmark's CPU-baseline leg call it; the
 * product library never does, and it shares no code, header or table with
 * the HIP path.
 *
 * Plain, slow and written to be checked by eye against the paper:
 *
 *   oracle_edt            exact squared EDT + nearest-site index, following
 *                         the four steps of the parallel banding algorithm
 *                         (Sec. III-C, Alg. 1) with one band per line:
 *                         step 1 nearest site in each row, step 2 proximate
 *                         sites of each column by a stack with a dominance
 *                         test, step 3 nearest-site query walking that stack,
 *                         step 4 steps 2-3 again along z.  All arithmetic is
 *                         int64.
 *   oracle_insert_points  point-cloud insertion (Sec. III-A): transform to
 *                         the map frame, discretize, set occupancy, skip
 *                         voxels the robot map occupies.
 *   oracle_insert_links   link voxel models placed by joint state (Sec. III-A,
 *                         Alg. 2 UpdateLinks/Insert).
 *   oracle_query_spheres  closest-obstacle extraction at sphere centres
 *                         (Alg. 2 ExtractClosestObstaclePose; Eq. dist).
 *
 * Readings where the paper is silent (all listed in the design notes):
 *   - tie rule: every step keeps the smaller coordinate on equal distance;
 *     with the passes in x, y, z order the final site is the smallest linear
 *     index among the equidistant occupied voxels;
 *   - empty map: d2 = INT32_MAX, site = -1; no sites outside the grid;
 *   - any nonzero occupancy byte is occupied;
 *   - float op order of insert / query is fixed (fmaf chain, correctly
 *     rounded divide and sqrt, floorf) so a device implementation can match
 *     bit for bit.  Build with -ffp-contract=off.
 *
 * Parity pins (tests/test_oracle_*.py): brute force over all sites on small
 * grids, closed forms for single sites and 1D rows, invariants (zero exactly
 * on occupied voxels, 1-Lipschitz, local optimality, sums of three squares).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define NONE (-1)

/* ------------------------------------------------------------------------ */
/* Step 1: nearest occupied voxel within a row (one "band" per row).        */
/* For each x, the nearest x' with occ != 0; on a tie the smaller x'.       */
/* ------------------------------------------------------------------------ */
static void row_nearest(const uint8_t* row, int n, int32_t* xs)
{
    /* left-to-right sweep: last site at or before x */
    int last = NONE;
    for (int x = 0; x < n; ++x) {
        if (row[x]) last = x;
        xs[x] = last;
    }
    /* right-to-left sweep: next site at or after x; keep the closer,
     * the left one on a tie */
    int next = NONE;
    for (int x = n - 1; x >= 0; --x) {
        if (row[x]) next = x;
        if (next != NONE) {
            if (xs[x] == NONE || (int64_t)(next - x) < (int64_t)(x - xs[x]))
                xs[x] = next;
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Steps 2 and 3 along one line of length n.                                */
/* Input: for each position p, g[p] = squared distance already accumulated */
/* in the other axes to that position's site, or -1 if it has no site.      */
/* Output: for each position q, the chosen site position best[q] (or NONE)  */
/* and the total squared distance dist[q] = g[best] + (q - best)^2.          */
/* ------------------------------------------------------------------------ */

/* value of site a's distance function at position q */
static int64_t f_at(int64_t a, int64_t ga, int64_t q)
{
    return ga + (q - a) * (q - a);
}

/* Is the site b (between a and c) dominated, i.e. is the stretch of the
 * line where b beats both a and c empty?  The boundary between a and b is
 * where f_a = f_b: q_ab = ((g_b+b^2) - (g_a+a^2)) / (2(b-a)).  b has no
 * stretch of its own iff q_bc <= q_ab; cross-multiplying by the positive
 * denominators keeps it exact. */
static int dominated(int64_t a, int64_t ga, int64_t b, int64_t gb, int64_t c, int64_t gc)
{
    int64_t ka = ga + a * a, kb = gb + b * b, kc = gc + c * c;
    return (kc - kb) * (b - a) <= (kb - ka) * (c - b);
}

static void line_envelope(const int64_t* g, int n, int32_t* best, int64_t* dist,
                          int32_t* stack /* scratch, n entries */)
{
    /* step 2: ComputeProximateSite -- sweep sites in order with a stack */
    int top = 0;
    for (int c = 0; c < n; ++c) {
        if (g[c] < 0) continue;
        while (top >= 2) {
            int a = stack[top - 2], b = stack[top - 1];
            if (dominated(a, g[a], b, g[b], c, g[c])) --top;
            else break;
        }
        stack[top++] = c;
    }
    /* step 3: QueryNearestSite -- for each position walk the stack while
     * the next proximate site is strictly closer (ties keep the smaller) */
    int k = 0;
    for (int q = 0; q < n; ++q) {
        if (top == 0) { best[q] = NONE; dist[q] = -1; continue; }
        while (k + 1 < top && f_at(stack[k + 1], g[stack[k + 1]], q) < f_at(stack[k], g[stack[k]], q))
            ++k;
        best[q] = stack[k];
        dist[q] = f_at(stack[k], g[stack[k]], q);
    }
}

/* ------------------------------------------------------------------------ */
/* Full 3D transform.  occ is [nz][ny][nx] with x fastest.                  */
/* d2 and site receive nx*ny*nz int32 values.  Returns 0, or -1 on bad args. */
/* nthreads <= 0 uses the OpenMP default; lines within a step are           */
/* independent, so the thread count does not change any value.             */
/* ------------------------------------------------------------------------ */
int oracle_edt(const uint8_t* occ, int nx, int ny, int nz, int32_t* d2,
               int32_t* site, int nthreads)
{
    if (!occ || !d2 || !site || nx < 1 || ny < 1 || nz < 1) return -1;
    const int64_t N = (int64_t)nx * ny * nz;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
    /* step 1 result: x' of the nearest site in the row (sx1); steps 2-3
     * result: the 2D site (sx2, sy2) of each voxel within its slice */
    int32_t* sx1 = (int32_t*)malloc(sizeof(int32_t) * N);
    int32_t* sx2 = (int32_t*)malloc(sizeof(int32_t) * N);
    int32_t* sy2 = (int32_t*)malloc(sizeof(int32_t) * N);
    if (!sx1 || !sx2 || !sy2) { free(sx1); free(sx2); free(sy2); return -1; }

    /* step 1, every row of every slice */
#pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < (int64_t)ny * nz; ++r)
        row_nearest(occ + r * nx, nx, sx1 + r * nx);

    /* steps 2-3 along y, for each column x of each slice z */
#pragma omp parallel
    {
        int64_t* g = (int64_t*)malloc(sizeof(int64_t) * ny);
        int64_t* dist = (int64_t*)malloc(sizeof(int64_t) * ny);
        int32_t* best = (int32_t*)malloc(sizeof(int32_t) * ny);
        int32_t* stk = (int32_t*)malloc(sizeof(int32_t) * ny);
#pragma omp for schedule(static)
        for (int64_t col = 0; col < (int64_t)nx * nz; ++col) {
            int64_t z = col / nx, x = col % nx;
            for (int y = 0; y < ny; ++y) {
                int32_t xp = sx1[x + (int64_t)nx * (y + (int64_t)ny * z)];
                g[y] = (xp == NONE) ? -1 : (x - xp) * (x - xp);
            }
            line_envelope(g, ny, best, dist, stk);
            for (int y = 0; y < ny; ++y) {
                int64_t i = x + (int64_t)nx * (y + (int64_t)ny * z);
                if (best[y] == NONE) { sx2[i] = NONE; sy2[i] = NONE; continue; }
                sx2[i] = sx1[x + (int64_t)nx * (best[y] + (int64_t)ny * z)];
                sy2[i] = best[y];
            }
        }
        free(g); free(dist); free(best); free(stk);
    }

    /* step 4: steps 2-3 along z for each (x, y) column, over the 2D sites */
#pragma omp parallel
    {
        int64_t* g = (int64_t*)malloc(sizeof(int64_t) * nz);
        int64_t* dist = (int64_t*)malloc(sizeof(int64_t) * nz);
        int32_t* best = (int32_t*)malloc(sizeof(int32_t) * nz);
        int32_t* stk = (int32_t*)malloc(sizeof(int32_t) * nz);
#pragma omp for schedule(static)
        for (int64_t col = 0; col < (int64_t)nx * ny; ++col) {
            int64_t y = col / nx, x = col % nx;
            for (int z = 0; z < nz; ++z) {
                int64_t i = x + (int64_t)nx * (y + (int64_t)ny * z);
                if (sx2[i] == NONE) g[z] = -1;
                else g[z] = (x - sx2[i]) * (x - sx2[i]) + (y - sy2[i]) * (y - sy2[i]);
            }
            line_envelope(g, nz, best, dist, stk);
            for (int z = 0; z < nz; ++z) {
                int64_t i = x + (int64_t)nx * (y + (int64_t)ny * z);
                if (best[z] == NONE) { d2[i] = INT32_MAX; site[i] = NONE; continue; }
                int64_t j = x + (int64_t)nx * (y + (int64_t)ny * best[z]);
                d2[i] = (int32_t)dist[z];
                site[i] = (int32_t)(sx2[j] + (int64_t)nx * (sy2[j] + (int64_t)ny * best[z]));
            }
        }
        free(g); free(dist); free(best); free(stk);
    }
    free(sx1); free(sx2); free(sy2);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Insertion (Sec. III-A).  T is a row-major 3x4 [R | t].                  */
/* ------------------------------------------------------------------------ */

/* map-frame coordinate: fixed fmaf chain R0*px + R1*py + R2*pz + t */
static float xform_row(const float* T, int r, float px, float py, float pz)
{
    return fmaf(T[4 * r + 2], pz, fmaf(T[4 * r + 1], py, fmaf(T[4 * r + 0], px, T[4 * r + 3])));
}

/* voxel coordinate u = (x - origin) / voxel; kept iff 0 <= u < n */
static int discretize(float x, float o, float v, int n, int* out)
{
    float u = (x - o) / v;
    if (!(u >= 0.0f && u < (float)n)) return 0;  /* also drops NaN */
    *out = (int)floorf(u);
    return 1;
}

static void insert_one(const float* T, const float* p, int nx, int ny, int nz,
                       const float* origin, float voxel, uint8_t* occ, const uint8_t* exclude)
{
    float x = xform_row(T, 0, p[0], p[1], p[2]);
    float y = xform_row(T, 1, p[0], p[1], p[2]);
    float z = xform_row(T, 2, p[0], p[1], p[2]);
    int ix, iy, iz;
    if (!discretize(x, origin[0], voxel, nx, &ix)) return;
    if (!discretize(y, origin[1], voxel, ny, &iy)) return;
    if (!discretize(z, origin[2], voxel, nz, &iz)) return;
    int64_t lin = ix + (int64_t)nx * (iy + (int64_t)ny * iz);
    if (exclude && exclude[lin]) return;   /* robot-part filtering */
    occ[lin] = 1;
}

void oracle_insert_points(int nx, int ny, int nz, const float* origin, float voxel,
                          uint8_t* occ, const float* pts, int64_t n, const float* T,
                          const uint8_t* exclude)
{
    for (int64_t i = 0; i < n; ++i)
        insert_one(T, pts + 3 * i, nx, ny, nz, origin, voxel, occ, exclude);
}

void oracle_insert_links(int nx, int ny, int nz, const float* origin, float voxel,
                         uint8_t* occ, const float* link_pts, const int32_t* link_off,
                         int n_links, const float* poses, uint64_t mask)
{
    for (int l = 0; l < n_links; ++l) {
        if (!((mask >> l) & 1u)) continue;
        for (int32_t i = link_off[l]; i < link_off[l + 1]; ++i)
            insert_one(poses + 12 * l, link_pts + 3 * (int64_t)i, nx, ny, nz, origin,
                       voxel, occ, NULL);
    }
}

/* ------------------------------------------------------------------------ */
/* Sphere query (Alg. 2 ExtractClosestObstaclePose; Eq. dist).              */
/* Each result is 16 x 4-byte words:                                        */
/*  0 d2  1 site  2..4 voxel  5 flags  6 dist_vox  7 x_c  8 clearance       */
/*  9..11 gradient  12..14 nearest obstacle centre O  15 zero               */
/* flags: 1 = centre outside the map, 2 = map empty.                        */
/* ------------------------------------------------------------------------ */
static float dist_at(const int32_t* d2, int64_t lin) { return sqrtf((float)d2[lin]); }

void oracle_query_spheres(int nx, int ny, int nz, const float* origin, float voxel,
                          const int32_t* d2, const int32_t* site, const float* centres,
                          const float* radii, int m, uint32_t* out)
{
    const int n3[3] = {nx, ny, nz};
    for (int i = 0; i < m; ++i) {
        uint32_t* o = out + 16 * (int64_t)i;
        union { float f; uint32_t u; int32_t s; } w[16];
        memset(w, 0, sizeof(w));
        const float* c = centres + 3 * i;
        float r = radii[i];
        int v[3], inside = 1;
        for (int a = 0; a < 3; ++a)
            if (!discretize(c[a], origin[a], voxel, n3[a], &v[a])) inside = 0;
        if (!inside) {
            /* outside the map: conservative distance 0, obstacle at centre */
            w[0].s = 0; w[1].s = NONE;
            w[2].s = w[3].s = w[4].s = -1;
            w[5].s = 1;
            w[6].f = 0.0f; w[7].f = 0.0f; w[8].f = -r;
            w[12].f = c[0]; w[13].f = c[1]; w[14].f = c[2];
        } else {
            int64_t lin = v[0] + (int64_t)nx * (v[1] + (int64_t)ny * v[2]);
            w[0].s = d2[lin]; w[1].s = site[lin];
            w[2].s = v[0]; w[3].s = v[1]; w[4].s = v[2];
            if (site[lin] == NONE) {
                w[5].s = 2;
                w[6].f = INFINITY; w[7].f = INFINITY; w[8].f = INFINITY;
                w[12].f = INFINITY; w[13].f = INFINITY; w[14].f = INFINITY;
            } else {
                int32_t s = site[lin];
                int sxyz[3] = {s % nx, (s / nx) % ny, s / (nx * ny)};
                float O[3], dd[3];
                for (int a = 0; a < 3; ++a) {
                    O[a] = fmaf((float)sxyz[a] + 0.5f, voxel, origin[a]);
                    dd[a] = O[a] - c[a];
                }
                float xc = sqrtf(fmaf(dd[2], dd[2], fmaf(dd[1], dd[1], dd[0] * dd[0])));
                w[6].f = dist_at(d2, lin);
                w[7].f = xc;
                w[8].f = xc - r;
                /* central difference of sqrt(d2) over +-1 voxel, one-sided
                 * at the borders, zero along an axis of length 1 */
                const int64_t stride[3] = {1, nx, (int64_t)nx * ny};
                for (int a = 0; a < 3; ++a) {
                    float g;
                    if (n3[a] == 1) g = 0.0f;
                    else if (v[a] == 0) g = dist_at(d2, lin + stride[a]) - dist_at(d2, lin);
                    else if (v[a] == n3[a] - 1) g = dist_at(d2, lin) - dist_at(d2, lin - stride[a]);
                    else g = 0.5f * (dist_at(d2, lin + stride[a]) - dist_at(d2, lin - stride[a]));
                    w[9 + a].f = g;
                }
                w[12].f = O[0]; w[13].f = O[1]; w[14].f = O[2];
            }
        }
        for (int k = 0; k < 16; ++k) o[k] = w[k].u;
    }
}

int oracle_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------------ */
/* Probabilistic occupancy (Sec. III-A: each point's voxel has its          */
/* occupancy updated as a Bayesian process).  Per frame, in log-odds:       */
/* a voxel holding at least one endpoint gets one hit update, a voxel that  */
/* some sensor ray crosses on its way to an endpoint (and that holds no     */
/* endpoint) gets one miss update, each clamped to [lmin, lmax]; the voxel  */
/* is occupied iff its log-odds exceed the threshold.  Only points whose    */
/* endpoint voxel lies in the map and is not excluded (and, given a keep   */
/* mask, that the filter kept) take part.                                   */
/*                                                                          */
/* The ray from the sensor voxel to the endpoint voxel is walked one voxel  */
/* at a time (the incremental traversal of Amanatides and Woo): in voxel    */
/* units a = (s - origin) / voxel, b = (p - origin) / voxel, d = b - a; an  */
/* axis with voxels left to cross has its next boundary crossing at         */
/* tmax = (boundary - a) / d, growing by 1 / |d| per crossing; every step   */
/* crosses on the axis with the smallest tmax (x before y before z on       */
/* ties) among those with voxels left, so the walk ends exactly on the      */
/* endpoint voxel after |dx| + |dy| + |dz| steps.  float32, one rounding    */
/* per operation in this order.                                             */
/* ------------------------------------------------------------------------ */
static inline int64_t lin3(int x, int y, int z, int nx, int ny)
{
    return x + (int64_t)nx * (y + (int64_t)ny * z);
}

/* Voxels from the start voxel to (excluding) the end voxel; returns the
 * number of steps, writes up to max_out voxels (x, y, z triples) of the
 * walk including the end voxel. */
int oracle_ray_walk(const float* a, const float* b, int32_t* out, int max_out)
{
    int cur[3], end[3], step[3], left[3];
    float tmax[3], tdel[3];
    int total = 0;
    for (int i = 0; i < 3; ++i) {
        cur[i] = (int)floorf(a[i]);
        end[i] = (int)floorf(b[i]);
        const float d = b[i] - a[i];
        step[i] = end[i] > cur[i] ? 1 : (end[i] < cur[i] ? -1 : 0);
        left[i] = step[i] > 0 ? end[i] - cur[i] : cur[i] - end[i];
        total += left[i];
        if (step[i] != 0) {
            const float bound = (float)(step[i] > 0 ? cur[i] + 1 : cur[i]);
            tmax[i] = (bound - a[i]) / d;
            tdel[i] = 1.0f / fabsf(d);
        } else {
            tmax[i] = INFINITY;
            tdel[i] = 0.0f;
        }
    }
    int n = 0;
    if (n < max_out) {
        out[3 * n + 0] = cur[0]; out[3 * n + 1] = cur[1]; out[3 * n + 2] = cur[2];
    }
    ++n;
    for (int k = 0; k < total; ++k) {
        int ax = -1;
        for (int i = 0; i < 3; ++i)
            if (left[i] > 0 && (ax < 0 || tmax[i] < tmax[ax])) ax = i;
        cur[ax] += step[ax];
        left[ax] -= 1;
        tmax[ax] = tmax[ax] + tdel[ax];
        if (n < max_out) {
            out[3 * n + 0] = cur[0]; out[3 * n + 1] = cur[1]; out[3 * n + 2] = cur[2];
        }
        ++n;
    }
    return total;
}

void oracle_update_logodds(int nx, int ny, int nz, const float* origin, float voxel,
                           int16_t* logodds, uint8_t* occ, const float* pts, int64_t n,
                           const float* T, const uint8_t* keep, const uint8_t* exclude, int hit,
                           int miss, int lmin, int lmax, int threshold)
{
    const int64_t nvox = (int64_t)nx * ny * nz;
    uint8_t* is_hit = (uint8_t*)calloc((size_t)nvox, 1);
    uint8_t* is_free = (uint8_t*)calloc((size_t)nvox, 1);
    const int n3[3] = {nx, ny, nz};
    /* sensor position in voxel units: the translation column of T */
    float a[3];
    for (int i = 0; i < 3; ++i) a[i] = (T[4 * i + 3] - origin[i]) / voxel;
    for (int64_t k = 0; k < n; ++k) {
        if (keep && !keep[k]) continue;   /* filtered out before insertion */
        const float* p = pts + 3 * k;
        float m[3], b[3];
        int e[3], ok = 1;
        for (int i = 0; i < 3; ++i) {
            m[i] = xform_row(T, i, p[0], p[1], p[2]);
            b[i] = (m[i] - origin[i]) / voxel;
            if (!(b[i] >= 0.0f && b[i] < (float)n3[i])) ok = 0;  /* drops NaN */
        }
        if (!ok) continue;
        for (int i = 0; i < 3; ++i) e[i] = (int)floorf(b[i]);
        const int64_t le = lin3(e[0], e[1], e[2], nx, ny);
        if (exclude && exclude[le]) continue;
        is_hit[le] = 1;
        /* a sensor farther than 2^16 voxels on an axis (or not finite)
         * walks no crossings */
        if (!(fabsf(a[0]) <= 65536.0f && fabsf(a[1]) <= 65536.0f && fabsf(a[2]) <= 65536.0f))
            continue;
        /* the walk's voxels before the endpoint are crossed: free */
        int cur[3], end[3], step[3], left[3], total = 0;
        float tmax[3], tdel[3];
        for (int i = 0; i < 3; ++i) {
            cur[i] = (int)floorf(a[i]);
            end[i] = e[i];
            const float d = b[i] - a[i];
            step[i] = end[i] > cur[i] ? 1 : (end[i] < cur[i] ? -1 : 0);
            left[i] = step[i] > 0 ? end[i] - cur[i] : cur[i] - end[i];
            total += left[i];
            if (step[i] != 0) {
                const float bound = (float)(step[i] > 0 ? cur[i] + 1 : cur[i]);
                tmax[i] = (bound - a[i]) / d;
                tdel[i] = 1.0f / fabsf(d);
            } else {
                tmax[i] = INFINITY;
                tdel[i] = 0.0f;
            }
        }
        for (int s = 0; s < total; ++s) {
            if (cur[0] >= 0 && cur[0] < nx && cur[1] >= 0 && cur[1] < ny && cur[2] >= 0 && cur[2] < nz)
                is_free[lin3(cur[0], cur[1], cur[2], nx, ny)] = 1;
            int ax = -1;
            for (int i = 0; i < 3; ++i)
                if (left[i] > 0 && (ax < 0 || tmax[i] < tmax[ax])) ax = i;
            cur[ax] += step[ax];
            left[ax] -= 1;
            tmax[ax] = tmax[ax] + tdel[ax];
        }
    }
    for (int64_t v = 0; v < nvox; ++v) {
        int l = logodds[v];
        if (is_hit[v]) {
            l += hit;
            if (l > lmax) l = lmax;
        } else if (is_free[v]) {
            l += miss;
            if (l < lmin) l = lmin;
        }
        logodds[v] = (int16_t)l;
        occ[v] = l > threshold ? 1 : 0;
    }
    free(is_hit);
    free(is_free);
}

/* ------------------------------------------------------------------------ */
/* Statistical outlier filtering of the raw cloud (Sec. III-A: points are   */
/* filtered by their Euclidean distance to their neighbours).  For every    */
/* finite point i:                                                          */
/*   s_ij = (dx*dx + dy*dy) + dz*dz of the float32 differences p_j - p_i;  */
/*   its neighbours are the other points with s_ij <= R*R, of which the k   */
/*   with the smallest s_ij count (fewer if there are fewer);               */
/*   d_i = (sum of sqrtf(s_ij) over them in ascending order + (k - m) * R)  */
/*         / k, m = number counted: a missing neighbour counts as R.        */
/* Over the finite points, mu and the sample standard deviation sigma of    */
/* d_i come from exact fixed-point sums (d_i in units of 2^-40, d_i^2 in    */
/* units of 2^-48); point i is kept iff it is finite and d_i <= mu +        */
/* alpha * sigma (double).  float32 with one rounding per operation for d_i.*/
/* ------------------------------------------------------------------------ */
static int finite3(const float* p)
{
    return isfinite(p[0]) && isfinite(p[1]) && isfinite(p[2]);
}

/* d_i of the listed points only (the same definition, O(m n)). */
static float outlier_mean_one(const float* pts, int64_t n, int64_t i, int k, float R);

void oracle_outlier_mean_dist(const float* pts, int64_t n, const int64_t* idx, int64_t m, int k,
                              float R, float* out)
{
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t t = 0; t < m; ++t) out[t] = outlier_mean_one(pts, n, idx[t], k, R);
}

static float outlier_mean_one(const float* pts, int64_t n, int64_t i, int k, float R)
{
    const float rr = R * R;
    const float* p = pts + 3 * i;
    if (!finite3(p)) return NAN;
    float best[64];
    int m = 0;
    for (int64_t j = 0; j < n; ++j) {
        if (j == i) continue;
        const float* q = pts + 3 * j;
        if (!finite3(q)) continue;
        const float dx = q[0] - p[0], dy = q[1] - p[1], dz = q[2] - p[2];
        const float s = (dx * dx + dy * dy) + dz * dz;
        if (!(s <= rr)) continue;
        if (m < k) {
            int t = m++;
            while (t > 0 && best[t - 1] > s) { best[t] = best[t - 1]; --t; }
            best[t] = s;
        } else if (s < best[k - 1]) {
            int t = k - 1;
            while (t > 0 && best[t - 1] > s) { best[t] = best[t - 1]; --t; }
            best[t] = s;
        }
    }
    float acc = 0.0f;
    for (int t = 0; t < m; ++t) acc = acc + sqrtf(best[t]);
    acc = acc + (float)(k - m) * R;
    return acc / (float)k;
}

void oracle_outlier_filter(const float* pts, int64_t n, int k, float R, double alpha,
                           uint8_t* keep, float* dmean, double* stats)
{
    int64_t S1 = 0, S2 = 0, cnt = 0;
#pragma omp parallel for schedule(dynamic, 64) reduction(+ : S1, S2, cnt)
    for (int64_t i = 0; i < n; ++i) {
        const float d = outlier_mean_one(pts, n, i, k, R);
        dmean[i] = d;
        if (!finite3(pts + 3 * i)) continue;
        const double dd = (double)d;
        S1 += (int64_t)rint(dd * 1099511627776.0);             /* 2^40 */
        S2 += (int64_t)rint(dd * dd * 281474976710656.0);      /* 2^48 */
        cnt += 1;
    }
    double mu = 0.0, sigma = 0.0;
    if (cnt > 0) mu = (double)S1 / 1099511627776.0 / (double)cnt;
    if (cnt > 1) {
        const double var = ((double)S2 / 281474976710656.0 - (double)cnt * mu * mu) / (double)(cnt - 1);
        sigma = var > 0.0 ? sqrt(var) : 0.0;
    }
    const double thr = mu + alpha * sigma;
    for (int64_t i = 0; i < n; ++i)
        keep[i] = finite3(pts + 3 * i) && (double)dmean[i] <= thr ? 1 : 0;
    stats[0] = mu;
    stats[1] = sigma;
    stats[2] = thr;
}

/* ------------------------------------------------------------------------ */
/* Jump flooding (the JFA of the paper's EDT comparison, Sec. IV / Table 2):*/
/* an approximate transform.  Seeds are the occupied voxels (site = own     */
/* index).  For step k = S/2, S/4, ..., 1 (S the smallest power of two      */
/* >= the largest axis), every voxel looks at the sites held by itself and  */
/* the 26 voxels at offsets in {-k, 0, k}^3 that lie in the grid, and keeps */
/* the one closest to it (squared voxel distance; the smaller linear index  */
/* on ties); all voxels read the previous step's sites.  d2 is the squared  */
/* distance to the final site (INT32_MAX / -1 where none was found).        */
/* ------------------------------------------------------------------------ */
int oracle_jfa(const uint8_t* occ, int nx, int ny, int nz, int32_t* d2, int32_t* site)
{
    const int64_t n = (int64_t)nx * ny * nz;
    int32_t* cur = (int32_t*)malloc((size_t)n * 4);
    int32_t* nxt = (int32_t*)malloc((size_t)n * 4);
    if (!cur || !nxt) { free(cur); free(nxt); return -1; }
    for (int64_t v = 0; v < n; ++v) cur[v] = occ[v] ? (int32_t)v : -1;
    int S = 1;
    while (S < nx || S < ny || S < nz) S <<= 1;
    for (int k = S / 2; k >= 1; k /= 2) {
#pragma omp parallel for schedule(static)
        for (int z = 0; z < nz; ++z)
            for (int y = 0; y < ny; ++y)
                for (int x = 0; x < nx; ++x) {
                    int32_t best = -1;
                    int64_t bd = 0;
                    for (int oz = -1; oz <= 1; ++oz)
                        for (int oy = -1; oy <= 1; ++oy)
                            for (int ox = -1; ox <= 1; ++ox) {
                                const int qx = x + ox * k, qy = y + oy * k, qz = z + oz * k;
                                if (qx < 0 || qx >= nx || qy < 0 || qy >= ny || qz < 0 || qz >= nz)
                                    continue;
                                const int32_t s = cur[qx + (int64_t)nx * (qy + (int64_t)ny * qz)];
                                if (s < 0) continue;
                                const int sx = s % nx, sy = (s / nx) % ny, sz = s / (nx * ny);
                                const int64_t dd = (int64_t)(sx - x) * (sx - x) +
                                                   (int64_t)(sy - y) * (sy - y) +
                                                   (int64_t)(sz - z) * (sz - z);
                                if (best < 0 || dd < bd || (dd == bd && s < best)) {
                                    best = s;
                                    bd = dd;
                                }
                            }
                    nxt[x + (int64_t)nx * (y + (int64_t)ny * z)] = best;
                }
        int32_t* t = cur;
        cur = nxt;
        nxt = t;
    }
    for (int64_t v = 0; v < n; ++v) {
        const int32_t s = cur[v];
        site[v] = s;
        if (s < 0) {
            d2[v] = INT32_MAX;
            continue;
        }
        const int x = (int)(v % nx), y = (int)((v / nx) % ny), z = (int)(v / ((int64_t)nx * ny));
        const int sx = s % nx, sy = (s / nx) % ny, sz = s / (nx * ny);
        d2[v] = (sx - x) * (sx - x) + (sy - y) * (sy - y) + (sz - z) * (sz - z);
    }
    free(cur);
    free(nxt);
    return 0;
}
