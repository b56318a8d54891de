/*
 * tsdf.h -- C ABI of the MI355X TSDF-mapping library (FeatSense TSDF path,
 * Gaal et al., arXiv 2310.05766, Sec. VI "TSDF Map Generation").
 *
 * The library integrates registered LiDAR scans, each taken at a given pose,
 * into a truncated signed distance field (Sec. VI), keeps a local map that
 * shifts after a movement threshold while writing what leaves it out and
 * loading what re-enters it (Sec. I), and keeps the global map (Sec. VII-C).
 *
 * Conventions shared by every call:
 *  - Fixed point. Positions are rounded to 1/1024 of a voxel in the global
 *    frame; signed distances are stored in the same unit.
 *  - Voxel storage (Sec. VI: a 16-bit value and a 16-bit weight per voxel).
 *    Two int16 arrays (SDF, weight), each [nx][ny][nz], z fastest, indexed
 *    by slot = floor_mod(g, dims) of the global voxel g (a ring buffer: a
 *    voxel that stays in the window never moves when the window shifts).
 *  - Streams. Every call on one map is ordered on that map's HIP stream.
 *  - Errors. Every call returns a tsdf_status; no exception crosses the ABI.
 *    TSDF_EINVAL leaves the map untouched. TSDF_EDEVICE poisons the map:
 *    afterwards only tsdf_map_destroy is accepted.
 *  - Threads. A map is used by one host thread at a time (TSDF_EBUSY if
 *    not); different maps may be used concurrently.
 */
#ifndef TSDF_H
#define TSDF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct tsdf_map tsdf_map; /* opaque: device arrays, scratch, host chunk store */

typedef enum {
    TSDF_OK = 0,
    TSDF_EINVAL = -1,  /* bad argument; nothing was changed */
    TSDF_ENOMEM = -2,  /* device or host allocation failed */
    TSDF_EDEVICE = -3, /* a HIP call failed; the map is poisoned */
    TSDF_ERANGE = -4,  /* a size exceeds what the library supports */
    TSDF_EBUSY = -5    /* the map is in use by another host thread */
} tsdf_status;

typedef enum { TSDF_PTR_HOST = 0, TSDF_PTR_DEVICE = 1 } tsdf_ptr_kind;

typedef struct {
    int32_t dims[3];     /* window size in voxels, each >= 1; nx*ny*nz < 2^31 */
    int32_t origin[3];   /* global voxel index of the window's min corner; the
                            window must lie within [-2^20, 2^20) voxels */
    double voxel_size_m; /* > 0 */
    int32_t tau_q10;     /* truncation tau in 1/1024-voxel units, 1..32767 */
    int32_t w_max;       /* weight cap of Eq. (2), 1..32767 */
} tsdf_map_desc;

typedef struct {
    int64_t points_in;      /* points passed in */
    int64_t points_valid;   /* finite, representable and not at the sensor */
    int64_t visits;         /* (ray, resident voxel) candidates */
    int64_t voxels_updated; /* voxels that received Eq. (1)/(2) this scan */
} tsdf_scan_stats;

/* Device scratch (bytes) a map with this descriptor uses for integration. */
size_t tsdf_scratch_bytes(const tsdf_map_desc *d);

/* Create a map whose SDF and weight arrays start at (0, 0) everywhere (w = 0
 * means unknown). hip_stream is a hipStream_t (NULL: the library creates its
 * own stream). The library owns every allocation. */
tsdf_status tsdf_map_create(const tsdf_map_desc *d, void *hip_stream, tsdf_map **out);

/* As tsdf_map_create, on caller-owned device memory: sdf_dev and w_dev hold
 * nx*ny*nz int16 each (layout above; the caller initialises them to a state
 * the method can reach, 0 <= w <= w_max and |sdf| <= tau_q10 per voxel, e.g.
 * all zero: other contents give unspecified values, never a fault), and
 * scratch_dev holds at least tsdf_scratch_bytes(d) bytes. They must outlive
 * the map; the library never frees them. */
tsdf_status tsdf_map_create_in(const tsdf_map_desc *d, void *sdf_dev, void *w_dev, void *scratch_dev,
                               size_t scratch_bytes, void *hip_stream, tsdf_map **out);

/* Waits for the map's stream and frees what the library owns. */
tsdf_status tsdf_map_destroy(tsdf_map *m);

/* Integrate one registered scan (Sec. VI: the min-tsdf step, then the
 * averaging step of Eq. (1) and Eq. (2) with one unit of weight per scan).
 *  xyz:   n_points x 3 float32, sensor frame, metres; a point with a
 *         non-finite coordinate is no return. Point i is row i (for an
 *         organised scan i = ring * columns + column); n_points < 2^32.
 *  kind:  TSDF_PTR_HOST -> copied into pinned staging before the call
 *         returns (the caller may reuse xyz at once); TSDF_PTR_DEVICE -> read
 *         on the map's stream (must stay valid until the stream passes it).
 *  world_T_sensor: row-major 4x4 float64 (host); only rows 0..2 are used and
 *         they must be finite, with the sensor position representable.
 *  stats: NULL -> the call returns without waiting for the GPU; otherwise
 *         the call waits and fills the counts of this scan. */
tsdf_status tsdf_integrate_scan(tsdf_map *m, const float *xyz, int64_t n_points, tsdf_ptr_kind kind,
                                const double world_T_sensor[16], tsdf_scan_stats *stats);

/* Move the window's min corner to new_origin (Sec. I: the local map is
 * shifted; what leaves it is written out, what re-enters it is loaded).
 * Leaving voxels go to the host chunk store (64^3-voxel chunks); entering
 * voxels come from it, or start at (0, 0). Synchronous. */
tsdf_status tsdf_shift(tsdf_map *m, const int32_t new_origin[3]);

/* Copy the global voxel box [lo, hi) to host arrays of (hi-lo) int16 each,
 * C order [x][y][z], z fastest: the resident value, else the stored value,
 * else (0, 0). Synchronous. */
tsdf_status tsdf_readback(tsdf_map *m, const int32_t lo[3], const int32_t hi[3], int16_t *sdf_out,
                          int16_t *w_out);

/* Batched form: scans that share a map are applied in array order, and the
 * result is bit-identical to calling tsdf_integrate_scan in that order. */
typedef struct {
    tsdf_map *map;
    const float *xyz;
    int64_t n_points;
    double pose[16];
} tsdf_scan_desc;

tsdf_status tsdf_integrate_batch(const tsdf_scan_desc *scans, int32_t count, tsdf_ptr_kind kind,
                                 void *hip_stream, tsdf_scan_stats *stats /* count entries, nullable */);

/* For callers that cannot allocate (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): tsdf_integrate_scan of
 * device points with no allocation and no graph. The batch engine's tables
 * and entry records live in one fixed device array of 64 MiB per GPU, held
 * by the library from its first use on that GPU until the process ends:
 * enough for one scan of 131,072 points at tau = 5 voxels on a 512 x 512 x
 * 256 window with the default tiling. Same arithmetic and result as
 * tsdf_integrate_scan.
 *  xyz_dev: device points (n_points x 3 float32), read on the map's stream.
 *  stats:   NULL -> returns without waiting; otherwise waits and fills them.
 * TSDF_ERANGE (map untouched) when the scan's tables would exceed the array;
 * TSDF_EINVAL for a map with interpolation or carving on (they allocate a
 * key volume) and for the arguments tsdf_integrate_scan rejects. Every call
 * on one GPU shares that GPU's array: calls that overlap on one GPU (maps
 * on different streams, or different host threads) race. */
tsdf_status tsdf_integrate_scan_noalloc(tsdf_map *m, const float *xyz_dev, int64_t n_points,
                                        const double world_T_sensor[16], tsdf_scan_stats *stats);

/* A batch runs on hip_stream (NULL: the first scan's map's stream), ordered
 * after earlier work on every map it touches, and later work on those maps
 * is ordered after it. The library keeps a batch engine (device tables,
 * staging) per stream; tsdf_batch_release frees the one of a stream after
 * waiting for it, and must be called before the caller destroys a stream it
 * passed here. (Destroying a map drops the engine of the map's own stream.) */
tsdf_status tsdf_batch_release(void *hip_stream);

/* Launch mode of every integration (process wide). on = 1 (the default):
 * each launch shape is captured once in a hipGraph (its five kernels, grid
 * sizes rounded up to powers of two) and replayed; the kernels read the
 * batch's real sizes from device memory. on = 0: direct kernel launches.
 * Results are identical in both modes. */
tsdf_status tsdf_set_graph_launch(int32_t on);

/* Stage timing of the batch engine of a stream (which exists once a batch
 * ran on it): while on, each batch launch is bracketed by HIP events on that
 * stream (and launched directly, not from a graph). Stages: 0 binning (ray
 * counts, runs, fill), 1 tile pass (candidates, minimum, Eq. (1)/(2)),
 * 2 per-scan counts, 3 the whole launch. _read waits for the stream and
 * returns the summed milliseconds and the number of launches. */
tsdf_status tsdf_batch_profile(void *hip_stream, int32_t on);
tsdf_status tsdf_batch_profile_read(void *hip_stream, int32_t stage, double *total_ms, int64_t *launches);

/* --- inspection and helpers (no method arithmetic beyond what is named) --- */

const char *tsdf_status_string(tsdf_status s);

/* Current window origin. */
tsdf_status tsdf_map_origin(const tsdf_map *m, int32_t origin[3]);

/* Device addresses of the SDF and weight arrays (layout above) and the
 * map's stream, for callers that wrap them (e.g. as tensors). */
tsdf_status tsdf_map_device_arrays(const tsdf_map *m, void **sdf_dev, void **w_dev, void **hip_stream);

/* Local-map recentre rule (the movement threshold of Sec. I): with o the
 * sensor position of world_T_sensor in fixed point, a shift is due when
 * |o - 1024 (origin + dims/2)|^2 > radius_q10^2; the new origin is the
 * chunk-grid point nearest the sensor voxel minus dims/2. force = 1 always
 * computes it (placement of the first window). *due is 1 when a shift is
 * due. Pure host arithmetic; the map is not changed. */
tsdf_status tsdf_recentre_origin(const tsdf_map *m, const double world_T_sensor[16], int64_t radius_q10,
                                 int32_t chunk, int32_t force, int32_t new_origin[3], int32_t *due);

/* Number of chunks and host bytes held by the map's chunk store. */
tsdf_status tsdf_store_info(const tsdf_map *m, int64_t *chunks, int64_t *bytes);

/* Wait until the map's stream has finished all queued work. */
tsdf_status tsdf_map_synchronize(tsdf_map *m);

/* --- per-kernel timing --------------------------------------------------
 * While profiling is on, every kernel launch of the map is bracketed by HIP
 * events recorded on the map's stream. tsdf_profile_enable(m, 1) waits for
 * the stream and discards earlier records; tsdf_profile_read waits for the
 * stream and returns the summed duration (ms) and the launch count of one
 * kernel since profiling was enabled. */
typedef enum {
    TSDF_KERNEL_BIN = 0,        /* ray binning by window tile (count, prefix, fill) */
    TSDF_KERNEL_TILE = 1,       /* per tile: walk, distances, LDS minimum, Eq. (1), Eq. (2) */
    TSDF_KERNEL_PACK = 2,       /* window -> staging (shift, readback) */
    TSDF_KERNEL_UNPACK = 3,     /* staging -> window (shift) */
    TSDF_KERNEL_COUNT = 8
} tsdf_kernel_id;

tsdf_status tsdf_profile_enable(tsdf_map *m, int32_t on);

/* Vertical interpolation between scan lines (Sec. VI, Eq. (3), Eq. (4)),
 * for the map's following scans: every band voxel also gives its value to
 * the voxels along the interpolation vector int = d x (d x up) (d: the ray,
 * up: the sensor's z axis), up to h = delta_z * len above and below the ray,
 * where len is the voxel's distance along the ray and
 * delta_z = tan(vfov_deg / hlines, in radians) (Eq. (3)). In fixed point:
 * d = rdiv(1024 D, r), up in 1/1024 units, delta_z in 1/2^20 units,
 * h = min(rdiv(delta_z len, 2^20), 65535), e = rdiv(h int, |int|); the
 * filled voxels of band voxel centre c are the floor-set of [c - e, c + e],
 * each receiving the band voxel's key; the per-scan minimum decides as for
 * the band. Rays with r >= 2^30 are not filled. vfov_deg = 0 turns it off;
 * vfov_deg / hlines must be below 45 degrees, and carving must be off
 * (else TSDF_EINVAL). The first
 * call that turns it on allocates an 8-byte key per voxel of the window
 * (TSDF_ENOMEM if that fails). Interpolating maps take their own
 * integration path (one thread per ray, 64-bit atomicMin on the key
 * volume); in tsdf_integrate_batch their scans run one by one, in order, on
 * their map's stream, ordered after the batch stream's earlier work and
 * before its later work. */
tsdf_status tsdf_map_set_interpolation(tsdf_map *m, double vfov_deg, int32_t hlines);
/* delta_z in 1/2^20 units, 0 when off. */
tsdf_status tsdf_map_get_interpolation(const tsdf_map *m, int64_t *delta_q20);

/* Free-space carving (a variant of the traversal: the ray traversed from the
 * sensor position p towards the scan point, Sec. VI), for the map's following
 * scans, on = 1 (0: off). Each ray longer than tau (r > tau) also walks the
 * segment [o, S] from the sensor to the start of its band; its voxels take
 * the ray's key exactly as band voxels do (s = clamp(rdiv((q - c) . D, r),
 * +-tau), mostly the truncated +tau), and the per-scan minimum and the merge
 * (Eq. (1), Eq. (2)) are unchanged. The band itself is unchanged; visits
 * count both segments, so the voxel where they meet counts twice. Any ray
 * the fixed point allows is walked exactly (|q|, |o| < 2^30). Not together
 * with vertical interpolation: TSDF_EINVAL when interpolation is on (and
 * tsdf_map_set_interpolation fails while carving is on). Carving maps take
 * the key-volume path described above (the first call that turns it on
 * allocates the 8-byte key per voxel; TSDF_ENOMEM if that fails), also in
 * tsdf_integrate_batch. */
tsdf_status tsdf_map_set_carving(tsdf_map *m, int32_t on);
/* 1 when carving is on, else 0. */
tsdf_status tsdf_map_get_carving(const tsdf_map *m, int32_t *on);

/* The number of 64-bit atomicMin operations the key-volume paths
 * (interpolation, carving) of this map have issued on its key volume since
 * the previous call (or since the key volume was allocated), then restarts
 * the count. These paths skip an atomic that could not lower the key it
 * read, so the count is at most the visits. Waits for the map's stream;
 * 0 for a map that never used the key volume. */
tsdf_status tsdf_map_key_atomics(tsdf_map *m, int64_t *issued);

/* Point-to-TSDF registration (the paper's stated next step, Sec. VIII;
 * HATSDF localises directly in its TSDF, Sec. I). A scan point p lands at
 * w = R p + t (float64, the integration's fma chain, metres); its residual
 * is the map's signed distance phi(w) in metres, trilinear between the 8
 * voxel centres around w, used only when all 8 are resident, observed and
 * not truncated (|sdf| < tau). Damped Gauss-Newton on sum phi^2:
 * (H + damping I) d = -J^T r with rows J = (grad phi, w x grad phi), then
 * R' = exp([theta]x) R, t' = exp([theta]x) t + rho for d = (rho, theta);
 * at most `iterations` steps (fewer when under 6 points remain or the
 * system is singular). The map is only read. Normal-equation sums are
 * formed in a fixed order (per block, then blocks in order), so results do
 * not depend on scheduling. Synchronous on the map's stream. */
typedef struct {
    int64_t points_used; /* at the returned pose */
    double cost;         /* sum of squared residuals there, m^2 */
    double last_step;    /* norm of the last step d */
    int32_t steps;       /* steps taken */
} tsdf_register_info;
tsdf_status tsdf_register_scan(tsdf_map *m, const float *xyz, int64_t n_points, tsdf_ptr_kind kind,
                               const double init_pose[16], int32_t iterations, double damping,
                               double pose_out[16], tsdf_register_info *info);
/* The normal equations at one pose: sums[0..20] = H (upper triangle, row-
 * major), sums[21..26] = J^T r, sums[27] = sum r^2, sums[28] = points used. */
tsdf_status tsdf_register_sums(tsdf_map *m, const float *xyz, int64_t n_points, tsdf_ptr_kind kind,
                               const double pose[16], double sums[29]);

/* Surface extraction for inspection: the zero level set of the resident
 * window inside the global voxel box [lo, hi) (which must lie inside the
 * window), as triangles of 9 floats each (three vertices, x y z in metres,
 * world frame) written to host memory tris. Marching tetrahedra: a cube is 8
 * observed (w > 0) voxel centres g + {0,1}^3 in the box, cut into the 6
 * tetrahedra around its diagonal from corner 0 to corner 7 (corner
 * k = (k & 1, k >> 1 & 1, k >> 2 & 1)); vertices with sdf < 0 are inside;
 * an edge from corner a to b crosses at t = s_a / (s_a - s_b) (float64),
 * the point ((g_a + 1/2) + t (g_b - g_a)) voxel_size rounded to float32.
 * Order: cubes by x, then y, then z; tetrahedra (0 1 3 7) (0 3 2 7)
 * (0 2 6 7) (0 6 4 7) (0 4 5 7) (0 5 1 7); one inside or one outside
 * vertex gives the triangle of its three edges in vertex order, two inside
 * (i0 < i1) and two outside (o0 < o1) give (i0o0, i0o1, i1o1) and
 * (i0o0, i1o1, i1o0). *n_tris gets the triangle count; tris = NULL (with
 * max_tris = 0) only counts; TSDF_ERANGE if max_tris is below the count.
 * Synchronous on the map's stream. */
tsdf_status tsdf_mesh(tsdf_map *m, const int32_t lo[3], const int32_t hi[3], float *tris, int64_t max_tris,
                      int64_t *n_tris);

/* Candidate-buffer tiling of the integration: the window is cut into tiles
 * of 2^log2_tile[a] voxels per axis (each in [2, 6], z at least 3,
 * 2^9..2^12 voxels per tile; a tile's candidate keys live in 8 bytes of LDS
 * per voxel), handled by tile_workgroups persistent workgroups (0: as many
 * as fit the device). log2_tile = {0, 0, 0}, the initial setting, lets the
 * library choose per call (16 x 16 x 8 tiles for tsdf_integrate_scan,
 * 8 x 8 x 8 for tsdf_integrate_batch, whose tiling is that of its first
 * scan's map); tsdf_map_get_tiling then reports {0, 0, 0}. The arithmetic,
 * and so every result, is the same for every tiling. */
tsdf_status tsdf_map_set_tiling(tsdf_map *m, const int32_t log2_tile[3], int32_t tile_workgroups);
tsdf_status tsdf_map_get_tiling(const tsdf_map *m, int32_t log2_tile[3], int32_t *tile_workgroups);

/* Block sizes of the integration kernels: bin_block threads per binning
 * block, one scan point each (128, 256 or 512; a block's rays share one LDS
 * table of tile counts), and tile_block threads per tile workgroup (256 or
 * 512; a workgroup holds about 32 KB of candidate keys per 256 threads).
 * 0 selects the default (256 for both); tsdf_map_get_blocks reports the
 * sizes in use. A batch uses its first scan's map's. The arithmetic, and so
 * every result, is the same for every choice; TSDF_EINVAL for other sizes. */
tsdf_status tsdf_map_set_blocks(tsdf_map *m, int32_t bin_block, int32_t tile_block);
tsdf_status tsdf_map_get_blocks(const tsdf_map *m, int32_t *bin_block, int32_t *tile_block);
tsdf_status tsdf_profile_read(tsdf_map *m, int32_t kernel, double *total_ms, int64_t *launches);
const char *tsdf_kernel_name(int32_t kernel);

#ifdef __cplusplus
}
#endif

#endif /* TSDF_H */
