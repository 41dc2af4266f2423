/*
 * edt.h -- C ABI of libedtmi.so: exact GPU distance maps for real-time
 * collision avoidance (Bedada & Palli, "Real Time Collision Avoidance with
 * GPU-Computed Distance Maps", arXiv 2407.02363) on AMD Instinct MI355X
 * (gfx950).
 *
 * One control cycle (Alg. 2): clear the maps, insert the robot's link voxel
 * models by joint state and the point cloud, compute the exact Euclidean
 * distance transform (Sec. III-C, Alg. 1), and extract the closest obstacle
 * at each bounding-sphere centre (ExtractClosestObstaclePose; Eq. dist).
 *
 * Conventions shared by every call:
 *   - Grid layout: a map is a dense array indexed lin = x + nx*(y + ny*z)
 *     (x fastest); 1 <= nx, ny, nz <= 1024.  origin is the map-frame position
 *     (metres) of the MIN corner of voxel (0,0,0); voxel is the edge length.
 *   - Pointers are DEVICE pointers unless stated otherwise.  The caller owns
 *     every buffer; no call allocates or frees device memory.
 *   - stream is a hipStream_t passed as void* (NULL = the null stream).  Every
 *     call only enqueues work on it and returns without synchronising, so
 *     the calls can be captured into a HIP graph.
 *   - Return value: EDT_OK (0) or a negative status.  Argument and shape
 *     errors are detected before anything is enqueued; nothing is launched
 *     then.  A failed launch returns EDT_ERR_HIP.  edt_last_error() gives a
 *     message for the last failure on the calling thread.  Faults inside a
 *     kernel surface at the caller's next synchronisation of the stream.
 */
#ifndef EDTMI_EDT_H
#define EDTMI_EDT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct edt_grid_t {
    int32_t nx, ny, nz;   /* voxels per axis, 1..1024 each */
    float origin[3];      /* metres, min corner of voxel (0,0,0) */
    float voxel;          /* edge length in metres, finite and > 0 */
} edt_grid_t;

/* One sphere query result (64 bytes). */
typedef struct edt_sphere_result_t {
    int32_t d2;           /* squared distance (voxels^2) at the centre's voxel */
    int32_t site;         /* linear index of the nearest occupied voxel */
    int32_t vox[3];       /* voxel containing the centre */
    int32_t flags;        /* EDT_Q_OUT_OF_MAP | EDT_Q_EMPTY, 0 if neither */
    float dist_vox;       /* sqrt(d2), voxels */
    float x_c;            /* ||O - C||, metres: Eq. dist with O the centre of
                             the nearest occupied voxel */
    float clearance;      /* x_c - radius, metres */
    float grad[3];        /* central difference of sqrt(d2) over +-1 voxel
                             (one-sided at the map border, 0 along an axis of
                             length 1), voxels per voxel */
    float nearest[3];     /* O, metres, map frame */
    float reserved;       /* 0 */
} edt_sphere_result_t;

enum {
    EDT_OK = 0,
    EDT_ERR_ARG = -1,         /* null pointer, negative count, bad flag */
    EDT_ERR_SHAPE = -2,       /* grid dimensions or voxel size out of range */
    EDT_ERR_WORKSPACE = -3,   /* workspace missing or too small */
    EDT_ERR_HIP = -4,         /* a HIP runtime call failed */
    EDT_ERR_UNSUPPORTED = -5  /* valid request this build does not handle */
};

enum { EDT_Q_OUT_OF_MAP = 1, EDT_Q_EMPTY = 2 };

/* Message for a status code (static string). */
const char* edt_status_string(int status);
/* Message of the last failed call on this thread ("" if none). */
const char* edt_last_error(void);
/* Library version string. */
const char* edt_version(void);

/*
 * edt_clear -- ClearMap of Alg. 2: set all nx*ny*nz bytes of occ to 0.
 * Uses a fill kernel (not a memset node), so it is safe to capture.
 */
int edt_clear(const edt_grid_t* grid, uint8_t* occ, void* stream);

/*
 * edt_insert_points -- insert a point cloud into an occupancy map
 * (Sec. III-A; Alg. 2 Insert(Point_Cloud)).
 *   pts       float32 [n][3], sensor frame.  NaN/inf or off-map points are
 *             dropped silently.
 *   n         number of points, >= 0 (0 enqueues nothing).
 *   T_map_sensor  float32 [12], device, row-major 3x4 [R | t] taking sensor
 *             coordinates to map coordinates.
 *   exclude   nullable uint8 [nx*ny*nz]: a point whose voxel is nonzero here
 *             (the robot's own map) is not inserted (robot-part filtering).
 * For each point, with fixed float32 op order:
 *   m_r = fmaf(T[4r+2], p.z, fmaf(T[4r+1], p.y, fmaf(T[4r], p.x, T[4r+3])))
 *   u_r = (m_r - origin[r]) / voxel   (correctly rounded)
 *   kept iff 0 <= u_r < n_r for r = x, y, z; voxel index floorf(u_r);
 *   occ[lin] = 1.
 * occ is OR-ed into (call edt_clear first for a fresh map).
 */
int edt_insert_points(const edt_grid_t* grid, uint8_t* occ, const float* pts, int64_t n,
                      const float* T_map_sensor, const uint8_t* exclude, void* stream);

/*
 * edt_jfa -- jump flooding, the approximate transform of the paper's EDT
 * comparison (Sec. IV, Table 2), for measuring its speed and its error
 * against edt_compute.  Seeds are the occupied voxels; for step k = S/2,
 * S/4, ..., 1 (S the smallest power of two >= the largest axis) every voxel
 * keeps, among the sites held by itself and the 26 voxels at offsets in
 * {-k, 0, k}^3 inside the grid, the one closest to it (squared voxel
 * distance, the smaller linear index on ties), all voxels reading the
 * previous step's sites.  Output as edt_compute: site is an occupied voxel
 * and d2 the exact squared distance to it, but the site need not be the
 * nearest one (d2 >= the exact transform's).  ws: device,
 * edt_jfa_workspace_bytes(grid) bytes (one int32 per voxel).
 */
size_t edt_jfa_workspace_bytes(const edt_grid_t* grid);
int edt_jfa(const edt_grid_t* grid, const uint8_t* occ, int32_t* d2, int32_t* site, void* ws,
            size_t ws_bytes, void* stream);

/*
 * Static-scene reuse (Exp. 4: one transform serves a static scene while the
 * arm moves).  edt_compute_cached keeps, in a caller-owned cache, a snapshot
 * of which voxels were occupied when d2 / site were last computed.  Each
 * call compares occ with it (occupied = any nonzero byte) and runs the
 * transform only if some voxel changed or the cache holds no result yet;
 * otherwise d2 and site are left as they are.  The decision is taken on the
 * device (the transform's kernels read a flag and return at once), so the
 * call never synchronises and replays correctly from a graph.
 *   cache  device, edt_cache_workspace_bytes(grid) bytes, zeroed by
 *          edt_cache_reset before the first call; one cache per (occ, d2,
 *          site) triple, and d2 / site must not be written between calls.
 * Results are identical to edt_compute.  Errors: as edt_compute, plus
 * EDT_ERR_WORKSPACE for a short cache.
 */
size_t edt_cache_workspace_bytes(const edt_grid_t* grid);
int edt_cache_reset(const edt_grid_t* grid, void* cache, size_t cache_bytes, void* stream);
int edt_compute_cached(const edt_grid_t* grid, const uint8_t* occ, int32_t* d2, int32_t* site,
                       void* cache, size_t cache_bytes, void* stream);

/*
 * Probabilistic occupancy (Sec. III-A: the occupancy of each point's voxel is
 * updated as a Bayesian process).  A persistent int16 log-odds grid (same
 * layout as occ) is updated once per frame:
 *   - a voxel holding at least one endpoint gets one hit update,
 *     L = min(L + hit, max);
 *   - a voxel that some sensor ray crosses on its way to an endpoint, and
 *     that holds no endpoint, gets one miss update, L = max(L + miss, min);
 *   - occ = 1 iff L > threshold (0 otherwise), ready for edt_compute.
 * Only points whose endpoint voxel lies in the map and is not set in
 * exclude take part (exclusion as in edt_insert_points).  The ray is walked
 * voxel by voxel from the sensor's voxel (the translation of T_map_sensor)
 * to the endpoint's: each step crosses the boundary with the smallest ray
 * parameter among the axes that still have voxels to cross (x before y
 * before z on ties), in float32 with one rounding per operation, so the
 * walk ends exactly on the endpoint voxel.  Voxels outside the map are
 * skipped; a sensor farther than 65536 voxels from the map origin on some
 * axis (or with a non-finite position) walks no crossings, its hits still
 * count.  Units: hundredths of a nat in the defaults below.
 */
typedef struct edt_logodds_t {
    int16_t hit;         /* added for an endpoint, e.g. 85 = ln(0.7 / 0.3) */
    int16_t miss;        /* added for a crossing, e.g. -41 = ln(0.4 / 0.6) */
    int16_t min, max;    /* clamp, e.g. -200 and 350 */
    int16_t threshold;   /* occupied iff log-odds > threshold, e.g. 0 */
    int16_t reserved;
} edt_logodds_t;

/* Workspace of the per-frame hit and crossing flags: 2 bytes per voxel.
 * Must be zero before the first update (edt_logodds_reset); every update
 * leaves it zero again. */
size_t edt_logodds_workspace_bytes(const edt_grid_t* grid);

/* log-odds = 0 (probability one half) everywhere and the workspace zeroed;
 * fill kernels only (graph-capturable). */
int edt_logodds_reset(const edt_grid_t* grid, int16_t* logodds, void* ws, size_t ws_bytes,
                      void* stream);

/* One frame: pts float32 [n][3] in the sensor frame, T_map_sensor device
 * float32 [12] (row-major 3x4), keep nullable uint8 [n] (0 = point filtered
 * out, e.g. by edt_outlier_filter), exclude nullable; logodds updated in
 * place, occ fully overwritten.  Errors: EDT_ERR_ARG (bad pointers,
 * min > max), EDT_ERR_WORKSPACE. */
int edt_update_logodds(const edt_grid_t* grid, int16_t* logodds, uint8_t* occ, const float* pts,
                       int64_t n, const float* T_map_sensor, const uint8_t* keep,
                       const uint8_t* exclude, const edt_logodds_t* params, void* ws,
                       size_t ws_bytes, void* stream);

/*
 * edt_outlier_filter -- statistical outlier filtering of a raw cloud before
 * insertion (Sec. III-A: points are filtered by their Euclidean distance to
 * their neighbours).  For every finite point i (all three coordinates
 * finite), in float32 with one rounding per operation:
 *   s_ij = (dx*dx + dy*dy) + dz*dz for the differences p_j - p_i, j != i;
 *   the neighbours are the finite j with s_ij <= radius*radius, of which the
 *   k closest count (m of them, m <= k);
 *   d_i = (sum of sqrtf(s_ij) over them in ascending order + (k - m) *
 *         radius) / k   -- a missing neighbour counts as radius.
 * mu and the sample standard deviation sigma of d_i over the finite points
 * come from exact fixed-point sums (d_i in units of 2^-40, d_i^2 in units of
 * 2^-48), so they do not depend on the order of accumulation; keep[i] = 1
 * iff point i is finite and d_i <= mu + alpha * sigma (double).  The
 * neighbour search is exact for coordinates within about 80 m of the
 * sensor origin (cells of 1.001 radius / 2).
 *   pts        device float32 [n][3], sensor frame; n <= EDT_OUTLIER_MAX_POINTS
 *   radius     metres, > 0; n * radius^2 must stay below 32,000 m^2 (and
 *              n * radius below 8e6 m) so that the exact sums cannot overflow
 *              (at 307,200 points: radius below 0.32 m; at the maximum count
 *              below 8.7 cm)
 *   k          1..16 neighbours
 *   keep       device uint8 [n] out
 *   mean_dist  device float32 [n] out (nullable): d_i, NaN for non-finite
 *   stats      device float64 [3] out (nullable): mu, sigma, threshold
 *   ws         device workspace of edt_outlier_workspace_bytes(n) bytes
 * Errors: EDT_ERR_ARG, EDT_ERR_WORKSPACE.  No synchronisation; fill
 * kernels only, graph-capturable.
 */
#define EDT_OUTLIER_MAX_POINTS 4194304
size_t edt_outlier_workspace_bytes(int64_t n_points);
int edt_outlier_filter(const float* pts, int64_t n, int32_t k, float radius, float alpha,
                       uint8_t* keep, float* mean_dist, double* stats, void* ws, size_t ws_bytes,
                       void* stream);

/*
 * edt_insert_links -- insert the robot's voxelized links placed by joint
 * state (Sec. III-A: offline link voxel models inserted according to the
 * joint state; Alg. 2 UpdateLinks/Insert; self-collision set O_L of
 * Eq. selfclink selected by link_mask).
 *   link_pts  float32 [P][3], link frames, all links back to back.
 *   link_off  HOST int32 [n_links+1]: points of link l are
 *             link_pts[link_off[l] .. link_off[l+1]).  Non-decreasing,
 *             link_off[0] = 0.
 *   n_links   1..64.
 *   link_poses float32 [n_links][12], device, row-major 3x4 link-to-map.
 *   link_mask bit l set = insert link l.
 * Same transform and discretisation as edt_insert_points; no exclusion.
 */
int edt_insert_links(const edt_grid_t* grid, uint8_t* occ, const float* link_pts,
                     const int32_t* link_off, int32_t n_links, const float* link_poses,
                     uint64_t link_mask, void* stream);

/*
 * edt_clear_insert_links_many -- ClearMap followed by UpdateLinks of Alg. 2
 * (as edt_clear, then edt_insert_links) for a batch of joint states that
 * share one grid -- the self map at every look-ahead state -- in two
 * launches for the whole batch.
 *   occ        HOST array of n_maps (1..EDT_BATCH_MAX) device pointers, read
 *              during the call: map j, nx*ny*nz bytes.  Maps must not overlap.
 *   link_poses float32 [n_maps][n_links][12] device: the link-to-map poses of
 *              state j at link_poses + 12 * n_links * j.
 *   link_pts, link_off, n_links, link_mask  as for edt_insert_links.
 *   gates      nullable DEVICE int32 [n_maps]: map j is cleared and filled
 *              only if gates[j] != 0 when the kernels run (else untouched).
 * Each map ends exactly as edt_clear + edt_insert_links leave it.
 */
int edt_clear_insert_links_many(const edt_grid_t* grid, uint8_t* const* occ, int32_t n_maps,
                                const float* link_pts, const int32_t* link_off, int32_t n_links,
                                const float* link_poses, uint64_t link_mask, const int32_t* gates,
                                void* stream);

/*
 * edt_workspace_bytes -- device workspace edt_compute needs for this grid
 * (0 for this version: the intermediate lives in the site output).
 */
size_t edt_workspace_bytes(const edt_grid_t* grid);

/*
 * edt_compute -- exact squared Euclidean distance transform with nearest
 * sites (Sec. III-C, Alg. 1).
 *   occ   uint8 [nx*ny*nz]; any nonzero byte is an occupied voxel (a site).
 *   d2    int32 [nx*ny*nz] out: min over sites s of |p - s|^2 (voxel units).
 *   site  int32 [nx*ny*nz] out: linear index of the nearest site; among
 *         equidistant sites the smallest linear index.
 *   If the map has no occupied voxel: d2 = INT32_MAX and site = -1
 *   everywhere.  Both outputs are fully overwritten (d2 also serves as
 *   scratch in between); they must not overlap occ or each other.  ws /
 *   ws_bytes: workspace of at least
 *   edt_workspace_bytes(grid) bytes (may be NULL when that is 0).
 */
int edt_compute(const edt_grid_t* grid, const uint8_t* occ, int32_t* d2, int32_t* site,
                void* ws, size_t ws_bytes, void* stream);

/*
 * Tile widths of the two EDT kernels: columns per work-group.  Each column
 * of a tile is split into group / tile bands, the m2 / m3 bands
 * of the paper's steps 2 and 3 (Sec. III-C): every band builds its own
 * envelope of proximate sites, neighbouring envelopes are merged, and every
 * band queries its own positions.  xy_tile is one of 16, 32, 64; z_tile one
 * of 8, 16, 32, 64; a tile whose work-group would need more local memory
 * than the device has is rejected with EDT_ERR_UNSUPPORTED.  Results do
 * not depend on the tiles.  The work-group sizes are xy_group and
 * z_group.
 */
typedef struct edt_tuning_t {
    int32_t xy_tile;
    int32_t z_tile;
    int32_t z_group;   /* threads per z work-group: 64, 128, 256 (0 = 256) or 512
                          with z_tile = 64;
                          z_tile <= z_group, bands per column = z_group / z_tile */
    int32_t xy_group;  /* threads per xy work-group: 64, 128, 256 (0 = 256) or 512
                          with xy_tile >= 32;
                          xy_tile <= xy_group, bands per column = xy_group / xy_tile.
                          xy_tile = xy_group and z_tile = z_group give one band per
                          line in both passes, the paper's naive m1 = m2 = m3 = 1 */
} edt_tuning_t;

/* Tiles edt_compute uses for this grid: the autotuner's choice if
 * edt_autotune ran for this shape in this process, else a heuristic. */
int edt_default_tuning(const edt_grid_t* grid, edt_tuning_t* out);

/* edt_compute with explicit tiles (NULL = edt_default_tuning). */
int edt_compute_tuned(const edt_grid_t* grid, const uint8_t* occ, int32_t* d2, int32_t* site,
                      const edt_tuning_t* tuning, void* stream);

/*
 * edt_compute_stage -- run one pass of edt_compute, for profiling and for
 * callers that pipeline the passes of several maps.
 *   stage EDT_STAGE_XY: steps 1-3 of Sec. III-C in every z slice; writes the
 *         2D nearest site of each voxel, packed x' | y' << 16 (0xFFFFFFFF if
 *         the slice is empty), into site.  With nx >= 256 it first writes
 *         per-row records of step 1 (12 bytes per 64 columns) into d2, as
 *         scratch; d2 holds nothing meaningful after this stage.
 *   stage EDT_STAGE_Z: step 4 (steps 2-3 along z); reads that packed form
 *         from site and overwrites d2 and site with the final result.
 *   stage EDT_STAGE_ALL: both, identical to edt_compute_tuned.
 *   tuning NULL = edt_default_tuning.
 */
enum { EDT_STAGE_XY = 1, EDT_STAGE_Z = 2, EDT_STAGE_ALL = 3 };
int edt_compute_stage(const edt_grid_t* grid, const uint8_t* occ, int32_t* d2, int32_t* site,
                      int stage, const edt_tuning_t* tuning, void* stream);

/*
 * edt_autotune -- pick the fastest tiles for this grid shape (the band
 * parameters m1, m2, m3 of Alg. 1 become tile widths here).  Runs every
 * valid (xy_tile, z_tile) pair `reps` times on occ (a representative map),
 * timing each pass with HIP events on `stream`, and records the winner in a
 * per-process cache keyed by (nx, ny, nz) that edt_compute and
 * edt_default_tuning consult.  Overwrites d2 and site.  Synchronises the
 * stream, so it must not be called while a graph is being captured.
 *   best     out (nullable): the chosen tiles.
 *   best_us  out (nullable): the chosen tiles' time for one full transform.
 */
int edt_autotune(const edt_grid_t* grid, const uint8_t* occ, int32_t* d2, int32_t* site,
                 int32_t reps, edt_tuning_t* best, float* best_us, void* stream);

/*
 * ---- batches of maps ----
 * Many maps of uneven size -- a fleet of robots, or one robot's maps at
 * several look-ahead states -- transformed in ONE persistent launch: the
 * xy tiles of every map, then the z tiles of every map, form a work queue
 * that resident work-groups drain; a map's z tiles wait (device-scope
 * acquire on a per-map counter) until all its xy tiles are released.
 * Results are identical to edt_compute on each map.
 */
#define EDT_BATCH_MAX 48

typedef struct edt_batch_map_t {
    edt_grid_t grid;      /* edt_compute_batched: every axis <= 512 voxels */
    const uint8_t* occ;   /* device, as for edt_compute */
    int32_t* d2;          /* device out */
    int32_t* site;        /* device out */
} edt_batch_map_t;

/*
 * edt_compute_many -- exact EDT (as edt_compute, Sec. III-C / Alg. 1) of
 * several maps in two launches: one xy launch over the tiles of every map,
 * then one z launch.  Maps may differ in shape (each axis up to 1024); a
 * map's work-groups start as soon as the previous map's free the GPU, so
 * each pass's slowest work-groups overlap other maps' work instead of
 * idling the GPU.  No workspace and no synchronisation; graph-capturable.
 *   maps    HOST array of n_maps (1..EDT_BATCH_MAX) descriptors, read during
 *           the call; buffers of different maps must not overlap.
 *   tuning  NULL = the tiles edt_compute would use for a grid with every
 *           map's largest extents; else as for edt_compute_tuned, valid for
 *           those extents.
 * Results are identical to one edt_compute per map.  Errors: argument and
 * shape errors as for edt_compute, EDT_ERR_UNSUPPORTED for tiles that do
 * not fit the largest map.
 */
int edt_compute_many(const edt_batch_map_t* maps, int32_t n_maps, const edt_tuning_t* tuning,
                     void* stream);

/*
 * edt_compute_many_gated -- edt_compute_many in which the device decides,
 * map by map, whether a map is transformed: for batches whose members are
 * chosen by earlier kernels (the look-ahead states whose predicted self
 * distances cannot be trusted, sdf_mlp_fallback), with no round trip to
 * the host in between.
 *   gates   DEVICE int32 [n_maps], or NULL (= edt_compute_many).  Map i is
 *           transformed only if gates[i] != 0; if it is 0, every work-group
 *           of map i returns at once and its d2 and site are left exactly as
 *           they were.  The kernels read gates when they run, so the values
 *           must be written before the call in stream order and must not
 *           change until it has finished; a captured graph reads them anew
 *           on every replay.
 * Everything else as for edt_compute_many.
 */
int edt_compute_many_gated(const edt_batch_map_t* maps, int32_t n_maps, const int32_t* gates,
                           const edt_tuning_t* tuning, void* stream);

/* Workspace bytes for a batch of n_maps (queue head, error flag, two
 * counters per map). */
size_t edt_batch_workspace_bytes(int32_t n_maps);

/*
 * edt_compute_batched -- exact EDT of every map of the batch.
 *   maps    HOST array of n_maps (1..EDT_BATCH_MAX) descriptors; buffers of
 *           different maps must not overlap.  The array is read during the
 *           call (its contents become kernel arguments), so a captured graph
 *           replays the same buffers.
 *   ws      device workspace of edt_batch_workspace_bytes(n_maps) bytes,
 *           zeroed by the call itself (a fill kernel, no memset node); two
 *           batches in flight at once need two workspaces.
 *   tuning  NULL = the batch autotuner's choice for this shape class, else
 *           xy_tile in {16, 32}, z_tile in {16, 32, 64} (z_group, xy_group ignored:
 *           batches use 256-thread work-groups), or xy_tile = z_tile = 64: the
 *           banded lean tiles of edt_compute (512-thread work-groups; every
 *           axis at most 512, nz at least 1).
 * Errors: EDT_ERR_UNSUPPORTED for an axis above 512 or tiles that do not
 * fit; argument errors as for edt_compute.
 */
int edt_compute_batched(const edt_batch_map_t* maps, int32_t n_maps, void* ws, size_t ws_bytes,
                        const edt_tuning_t* tuning, void* stream);

/*
 * edt_compute_batched_noalloc -- edt_compute_batched for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): the same kernels and results, with the
 * batch's workspace taken from a 512-byte array that the library holds on
 * every GPU it runs on until the process ends.  The call allocates nothing:
 * no hipMalloc, hipFree or allocating library routine.
 *   maps, n_maps, tuning  as for edt_compute_batched (n_maps <= EDT_BATCH_MAX,
 *           the limit of the array; more maps fail with EDT_ERR_ARG).
 *   timed_out  nullable DEVICE int32: after the batch, 1 if a wait gave up
 *           (as edt_batch_status reports), else 0; written in stream order.
 * Every call on one GPU shares that GPU's array, which keeps the last call's
 * contents (the call clears what must start at zero): calls that overlap on
 * one GPU race.  The first call on a device looks up the array's address
 * there (hipGetSymbolAddress); make it outside graph capture.
 */
int edt_compute_batched_noalloc(const edt_batch_map_t* maps, int32_t n_maps, const edt_tuning_t* tuning,
                                int32_t* timed_out, void* stream);

/* Synchronises the stream and reports whether a batch launch that used ws
 * gave up waiting for a map's xy tiles (*timed_out = 1: that map's result
 * is incomplete).  Never expected; a guard against a stuck queue. */
int edt_batch_status(const void* ws, int32_t* timed_out, void* stream);

/* Times every batch tile pair on this batch (reps launches each, HIP
 * events), caches the fastest for batches with the same count and maximum
 * dimensions, and leaves its result in the outputs.  Synchronises. */
int edt_autotune_batched(const edt_batch_map_t* maps, int32_t n_maps, void* ws, size_t ws_bytes,
                         int32_t reps, edt_tuning_t* best, float* best_us, void* stream);

/*
 * The tile choices of edt_autotune and edt_autotune_batched are cached in the
 * process per device architecture (the part of the HIP architecture name
 * before any ':', e.g. "gfx950") and shape: edt_compute and
 * edt_compute_many use the cached tiles of a map's shape on a device of that
 * architecture, edt_compute_batched those of a batch's map count and largest
 * extents.  The cache can be written to a text file and read back by a later
 * process, so that autotuning runs once per machine type and shape:
 *   edt_tuning_cache_save  writes every entry to path (overwriting it);
 *                          returns the number of entries written.
 *   edt_tuning_cache_load  adds the file's entries to the cache (an entry for
 *                          the same architecture and shape is replaced);
 *                          returns the number of entries read.  A file that
 *                          is not a cache, or any line that is not a valid
 *                          entry (tiles the library cannot launch for that
 *                          shape), fails with EDT_ERR_ARG and adds nothing.
 *   edt_tuning_cache_clear forgets every entry (the heuristic tiles apply).
 * File format: the line "edtmi tuning cache v1", then one entry per line,
 *   single <arch> <nx> <ny> <nz> xy <xy_tile> <xy_group> z <z_tile> <z_group>
 *   batch <arch> <maps> <nx> <ny> <nz> xy <xy_tile> <xy_group> z <z_tile> <z_group>
 * blank lines and lines starting with '#' ignored.  Host-only calls; no GPU
 * is needed to save or load.
 */
int edt_tuning_cache_save(const char* path);
int edt_tuning_cache_load(const char* path);
int edt_tuning_cache_clear(void);

/*
 * edt_query_spheres -- closest obstacle at bounding-sphere centres
 * (Alg. 2 ExtractClosestObstaclePose; task variable x_c of Eq. dist and the
 * constraint x_c >= radius of Eq. ref).
 *   d2, site   outputs of edt_compute for this grid.
 *   centres    float32 [m][3], map frame, metres.
 *   radii      float32 [m].
 *   out        edt_sphere_result_t [m], device.
 * A centre outside the map gets flags EDT_Q_OUT_OF_MAP and a conservative
 * distance of 0 (d2 = 0, site = -1, vox = -1, x_c = 0, clearance = -radius,
 * nearest = the centre).  On an empty map flags = EDT_Q_EMPTY and the
 * distances are +inf.  Float op order is fixed: O_a = fmaf(s_a + 0.5, voxel,
 * origin_a); x_c = sqrtf(fmaf(dz, dz, fmaf(dy, dy, dx*dx))) with d = O - C.
 */
int edt_query_spheres(const edt_grid_t* grid, const int32_t* d2, const int32_t* site,
                      const float* centres, const float* radii, int32_t m,
                      edt_sphere_result_t* out, void* stream);

/*
 * edt_query_spheres_many -- edt_query_spheres for every map of a batch in one
 * launch (the bounding spheres of every look-ahead state, or of every map of
 * a batched cycle).
 *   maps      HOST array of n_maps (1..EDT_BATCH_MAX) descriptors, read during
 *             the call: grid, d2 and site of map j (occ unused).
 *   centres, radii, out  HOST arrays of n_maps device pointers: map j's
 *             float32 [m[j]][3] centres, float32 [m[j]] radii and
 *             edt_sphere_result_t [m[j]] results.
 *   m         HOST int32 [n_maps]: spheres per map (0 allowed).
 * Record k of map j is exactly what edt_query_spheres gives for map j,
 * centre k.
 */
int edt_query_spheres_many(const edt_batch_map_t* maps, int32_t n_maps, const float* const* centres,
                           const float* const* radii, const int32_t* m, edt_sphere_result_t* const* out,
                           void* stream);

/*
 * edt_clear_insert_points_many -- ClearMap followed by Insert(Point_Cloud) of
 * Alg. 2 (as edt_clear, then edt_insert_points without an exclusion mask)
 * for every map of a batch, each with its own grid, cloud and sensor pose, in
 * two launches for the whole batch.
 *   grids         HOST array of n_maps (1..EDT_BATCH_MAX) grids.
 *   occ           HOST array of n_maps device pointers: map j's occupancy.
 *   pts, T_map_sensor  HOST arrays of device pointers: map j's float32
 *                 [n_pts[j]][3] cloud (sensor frame) and float32 [12] pose.
 *   n_pts         HOST int64 [n_maps]: points per map (0 allowed).
 * Each map ends exactly as edt_clear + edt_insert_points leave it.  Maps must
 * not overlap.
 */
int edt_clear_insert_points_many(const edt_grid_t* grids, uint8_t* const* occ, int32_t n_maps,
                                 const float* const* pts, const int64_t* n_pts,
                                 const float* const* T_map_sensor, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* EDTMI_EDT_H */
