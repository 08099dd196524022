/*
 * vrt.h -- C ABI of the MI355X voxel ray tracer for dynamic line sets.
 *
 * The library implements the per-frame path of arXiv 2510.09081 (Section 3):
 *   vrt_voxelize  conservative capsule voxelization of every segment into a
 *                 grid, per-voxel fragment count and occupancy in one packed
 *                 32-bit word, and the averaging occupancy pyramid
 *                 (Section 3.1, Alg. 1-3);
 *   vrt_cull      erosion, camera-visibility culling and the culling pyramid
 *                 (Section 3.2), then the exclusive scan of visible counts and
 *                 the second voxelization pass that writes per-voxel segment
 *                 lists (Section 3.3, voxelize-cull-scan-voxelize);
 *   vrt_trace     one primary ray per pixel through the culling pyramid and the
 *                 grid, exact ray-capsule hits with clip planes, the in-voxel
 *                 acceptance rule, opaque first hit or sorted front-to-back
 *                 compositing (Section 3.5).
 *
 * Conventions
 *   - Pointers named "device" are HIP device memory owned by the caller; they
 *     are only read or written by work enqueued on the given stream and must
 *     stay valid until that work completes.  Struct arguments are read on the
 *     host before the call returns.
 *   - Positions are quantized to 1/256 voxel (int32, |q| < 2^20) relative to
 *     the grid corner; the radius likewise.  Voxel membership, counts, culling
 *     and list building are exact integer computations; the per-fragment
 *     occupancy quantum is a fixed binary32 sequence.
 *   - A segment is the pair of consecutive vertices (v_i, v_{i+1}) inside one
 *     polyline; its id is i, the global index of its first vertex.
 *   - The acceleration structure lives in arenas owned by the context and
 *     sized at creation; no entry point allocates memory after vrt_create.
 *     One context serves one stream at a time; contexts are independent.
 *   - Status: 0 is success.  Argument errors are detected on the host before
 *     anything is enqueued.  Errors that depend on device data (range,
 *     capacity, count overflow) latch in a device status word, are reported
 *     by vrt_frame_status, and leave that frame's outputs undefined.
 */
#ifndef VRT_H
#define VRT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t vrt_status;

#define VRT_OK 0
#define VRT_ERR_INVALID_ARG 1    /* null pointer, bad size, bad enum, dims not a multiple of 8 ... */
#define VRT_ERR_RANGE 2          /* coordinates beyond the fixed-point range, segment longer than 256 voxels */
#define VRT_ERR_NOT_BUILT 3      /* vrt_cull before vrt_voxelize, vrt_trace before vrt_cull */
#define VRT_ERR_CAPACITY 4       /* listed fragments exceed max_fragments */
#define VRT_ERR_COUNT_OVERFLOW 5 /* more than 65535 fragments in one voxel (16-bit count field) */
#define VRT_ERR_HIP 6            /* a HIP runtime call failed; see vrt_last_hip_error */

#define VRT_CULL_NONE 0   /* every occupied voxel is visible (voxelize-scan-voxelize) */
#define VRT_CULL_OPAQUE 1 /* hidden behind one blocking voxel */
#define VRT_CULL_ALPHA 2  /* hidden behind as many blocking voxels as alpha layers reach tau */

#define VRT_TRACE_OPAQUE 0
#define VRT_TRACE_TRANSPARENT 1

#define VRT_FORM_PLAIN 0 /* the tracer reads the int32 vertex records */
#define VRT_FORM_FP16 1  /* the tracer reads per-segment FP16 records (brick-relative endpoints) */

typedef struct vrt_ctx vrt_ctx;

/* Capacities fixed at creation (Section 3.3: the lists are sized by the scan,
 * so a capacity bounds them without a host round trip). */
typedef struct {
    int64_t max_vertices;  /* largest n_vertices accepted by vrt_voxelize */
    int64_t max_fragments; /* capacity of the segment-id array (listed fragments) */
    int32_t max_dim;       /* largest grid dimension; multiple of 8, <= 1024 */
    int32_t device;        /* HIP device ordinal the arenas live on */
    int64_t max_pixels;    /* largest width * height accepted by vrt_trace */
    int32_t form;          /* VRT_FORM_PLAIN or VRT_FORM_FP16: the segment records the tracer reads.  FP16:
                              each segment stores its endpoints as binary16 offsets (voxel units) from the centre
                              of the 8^3 brick holding its midpoint, 16-bit fixed-point clip normals and int16 brick
                              coordinates (32 B per segment instead of two 32-B vertex records); intersection
                              and compositing stay binary32 and voxel membership stays exact int32.  Offsets
                              are exact while |offset| < 8 voxels; a segment with a longer offset is
                              read from its plain vertex records instead. */
    int32_t reserved;
} vrt_desc;

/* Membership of a segment's voxels.  VRT_VOX_CAPSULE is the paper's
 * conservative capsule voxelization (Section 3.1, Alg. 1 with the projected
 * radius that is conservative in 3D); the other two are the comparison
 * voxelizers of Section 4.1 (Table 2), kept for measurement: their lists are
 * not conservative for the capsules (thin) or much longer (AABB), and the
 * image they trace is not the capsule image. */
#define VRT_VOX_CAPSULE 0
#define VRT_VOX_THIN 2 /* the voxels whose open interior the segment meets, plus its endpoints' cells (a 3D DDA) */
#define VRT_VOX_AABB 3 /* every voxel touching the capsule's bounding box */

/* A set of polylines with one radius (Section 3.1: capsules of uniform radius
 * per polyline; polylines neither branch nor loop, Section 3.3). */
typedef struct {
    const float *xyz;            /* device, [3 * n_vertices], world units, xyz interleaved */
    const int32_t *poly_offsets; /* device, [n_polylines + 1], polyline p = [off[p], off[p+1]); off[0] = 0,
                                    off[n_polylines] = n_vertices, non-decreasing */
    int64_t n_vertices;
    int64_t n_polylines;
    float radius;                /* capsule radius, world units, >= 0 */
    float alpha_default;         /* transparent traces: opacity of every segment when rgba is NULL, in (0, 1];
                                    0 = the camera's alpha */
    const float *rgba;           /* device, [4 * n_vertices], 16-byte aligned, or NULL: colour and opacity of
                                    segment i (the one starting at vertex i) at rgba[4 i .. 4 i + 3]; rows of
                                    polyline end vertices are unused.  Read by vrt_trace (keep it valid until
                                    the frame's traces complete); opacity is clamped to [0, 1].  NULL: colour =
                                    |unit tangent| */
    int32_t voxelizer;           /* VRT_VOX_*; 0 = VRT_VOX_CAPSULE */
    int32_t reserved;            /* 0 */
} vrt_lines;

/* Axis-aligned grid of isotropic voxels; voxel (x,y,z) covers
 * origin + voxel_size * [x, x+1) x [y, y+1) x [z, z+1). */
typedef struct {
    float origin[3];
    float voxel_size; /* > 0 */
    int32_t dims[3];  /* each a multiple of 8, 8 <= dims <= max_dim */
} vrt_grid;

/* View for culling (Section 3.2). */
typedef struct {
    float eye[3];      /* world units */
    int32_t cull_mode; /* VRT_CULL_* */
    float alpha;       /* VRT_CULL_ALPHA: per-layer opacity in (0, 1] */
    float tau;         /* VRT_CULL_ALPHA: transmittance threshold in (0, 1) */
} vrt_view;

/* Pinhole camera (Section 3.5: one ray per pixel). */
typedef struct {
    float eye[3], target[3], up[3]; /* world units; up not parallel to target - eye */
    float fovy_deg;                 /* vertical field of view, (0, 180) */
    int32_t width, height;          /* pixels, >= 1 */
    int32_t mode;                   /* VRT_TRACE_* */
    float alpha;                    /* transparent: per-hit opacity in (0, 1] (segments without their own
                                       colour, when the lines give no alpha_default) */
    float tau;                      /* transparent: stop once transmittance < tau */
} vrt_camera;

/* Output image, row 0 at the top, pixel (x, y) at index y * width + x. */
typedef struct {
    float *rgba;       /* device, [4 * W * H]; opaque: colour of the first hit, alpha 1;
                          transparent: premultiplied composite, A = 1 - transmittance; 0 on a miss */
    float *depth;      /* device, [W * H] or NULL; world distance to the first hit, +inf on a miss */
    int32_t *first_id; /* device, [W * H] or NULL; segment id of the first hit, -1 on a miss */
} vrt_image;

/* Per-frame totals; filled by vrt_frame_status. */
typedef struct {
    vrt_status device_status; /* first latched device error of the frame, or VRT_OK */
    int64_t n_fragments;      /* pass-1 fragments: sum over segments of |voxel set| */
    int64_t n_listed;         /* fragments written to lists (visible voxels only) */
    int64_t n_bricks;         /* occupied 8^3 bricks */
    int64_t required_fragments; /* capacity the frame needed (== n_listed) */
    int64_t n_occupied;       /* occupied voxels (fragment count > 0) */
    int64_t n_visible;        /* voxels the last vrt_cull left visible (those with a list) */
} vrt_frame_info;

/* Read-only device views of the acceleration structure for inspection.
 * Layout: brick b = (bz * NBy + by) * NBx + bx with NB = dims / 8; level-0
 * per-voxel arrays hold 512 entries per brick (x fastest inside the brick),
 * level-1 arrays 64 (4^3) and level-2 arrays 8 (2^3) per brick; level-3
 * arrays one entry per brick (dense over all bricks).  Only bricks listed in
 * brick_list are defined at levels 0-2.  Levels >= 4 are dense x-fastest grids
 * of size ceil(dims / 2^L), stored back to back from level 4 upwards. */
typedef struct {
    int32_t dims[3];
    int32_t n_levels;            /* levels 0 .. n_levels-1; the last is 1^3 */
    int32_t n_bricks;            /* occupied bricks (copied from the device; synchronizes) */
    const int32_t *brick_list;   /* [n_bricks] ascending brick indices */
    const uint32_t *words;       /* level 0: count (low 16 bits) + occupancy sum (high 16 bits) */
    const uint16_t *occ[4];      /* occupancy levels 0..3 (1/256 units) */
    const uint16_t *occ_hi;      /* occupancy levels >= 4 */
    const uint8_t *blocking;     /* level 0: eroded occupancy is full */
    const uint8_t *vis[4];       /* culling levels 0..3 */
    const uint8_t *vis_hi;       /* culling levels >= 4 */
    const uint32_t *list_end;    /* level 0: end of the voxel's list in ids (start = end - count) */
    const uint32_t *ids;         /* [n_listed] segment ids */
    const float *lit;            /* level 0: voxel-space shading of the visible voxels (after vrt_shade) */
} vrt_as_view;

/* Creates a context on desc->device and allocates every arena.
 * Errors: VRT_ERR_INVALID_ARG, VRT_ERR_HIP (allocation failure). */
vrt_status vrt_create(const vrt_desc *desc, vrt_ctx **out);

/* Frees every arena; waits for outstanding work of the context. */
vrt_status vrt_destroy(vrt_ctx *ctx);

/* Section 3.1: quantizes the vertices, derives the clip-plane normals (the
 * central-difference tangent at interior vertices), clears what the previous
 * frame wrote, and runs voxelization pass 1 (count + occupancy, one packed
 * atomic per fragment) and the occupancy pyramid.  stream: hipStream_t. */
vrt_status vrt_voxelize(vrt_ctx *ctx, const vrt_lines *lines, const vrt_grid *grid, void *stream);

/* Sections 3.2 and 3.3: erosion and blocking flags, one culling ray per
 * occupied voxel toward view->eye, the culling pyramid, the exclusive scan of
 * visible counts (8^3 bricks in order, x fastest inside a brick) and pass 2,
 * which writes each segment's id into the lists of its visible voxels.
 * Requires a preceding vrt_voxelize on the same context. */
vrt_status vrt_cull(vrt_ctx *ctx, const vrt_view *view, void *stream);

/* Section 3.3 leaves the order of the segment ids inside a voxel's list
 * undefined, and the slot atomics of pass 2 vary it from run to run.  This
 * sorts every visible voxel's list ascending by segment id (the canonical
 * order), after which the id array is a deterministic function of the frame
 * -- for a static line set built once and traced many times, or to compare
 * lists byte for byte.  Lists are rebuilt (unsorted) by the next vrt_cull.
 * Requires a preceding vrt_cull; does nothing after a capacity overflow.
 * Errors: VRT_ERR_INVALID_ARG, VRT_ERR_NOT_BUILT, VRT_ERR_HIP. */
vrt_status vrt_sort_lists(vrt_ctx *ctx, void *stream);

/* Voxel-space shading (Section 3.4): after vrt_cull, computes for every
 * visible voxel
 *   AO  = mean over n_cones cones of the transmittance 1 - a, where a
 *         accumulates front to back (a += (1 - a) o_j) the occupancy o_j of
 *         the level-j pyramid cell holding the point 2^j voxels from the
 *         voxel centre along the cone's direction, j = 1..n_samples; the
 *         directions are the points of a Fibonacci sphere (heights evenly
 *         spaced, longitudes advancing by the golden angle) rounded to
 *         1/256 voxel;
 *   S   = the product of (1 - occupancy) over the voxels a ray from the
 *         voxel centre toward the light enters before it leaves the grid
 *         (exact integer walk, tied axes step together);
 *   lit = AO * (ambient + (1 - ambient) * S),
 * and the following vrt_trace calls scale each hit's colour by lit of the
 * voxel holding the hit point (opacity unchanged).  The next vrt_cull (new
 * visibility) turns shading off until vrt_shade runs again.
 * enable = 0 turns it off without computing anything.
 * Errors: VRT_ERR_INVALID_ARG (n_cones outside 1..64, n_samples outside
 * 1..6 or not below the pyramid's level count, ambient outside [0, 1], a
 * zero or non-finite light direction), VRT_ERR_NOT_BUILT before vrt_cull. */
typedef struct {
    float light_dir[3]; /* direction toward the light, world axes (normalized here) */
    int32_t n_cones;    /* ambient-occlusion cones, 1..64 (16 by default) */
    int32_t n_samples;  /* samples per cone, 1..6 (4: out to 16 voxels) */
    float ambient;      /* weight of the unshadowed term, [0, 1] */
    int32_t enable;     /* 0: unshaded colours */
    int32_t reserved;   /* 0 */
} vrt_shading;

vrt_status vrt_shade(vrt_ctx *ctx, const vrt_shading *shading, void *stream);

/* Section 3.5: traces one ray per pixel and writes the image.  Requires a
 * preceding vrt_cull.  The ray origin is cam->eye quantized like the
 * vertices; directions are a fixed binary32 function of the camera. */
vrt_status vrt_trace(vrt_ctx *ctx, const vrt_camera *cam, const vrt_image *out, void *stream);

/* Per-frame graph (the replay pattern for dynamic line sets): captures
 * one frame -- vrt_voxelize, then for each pass i vrt_cull(views[i]) and
 * vrt_trace(cams[i], imgs[i]) -- into a HIP graph on a private capture stream.
 * Each vrt_graph_launch replays the whole frame on `stream` with no host work;
 * it reads the vertex and offset buffers and writes the images at the
 * addresses given here, so a dynamic line set updates those buffers in place
 * between launches (same vertex and polyline counts).  The context must
 * outlive the graph and must not be used by other calls while a replay runs.
 * Errors: VRT_ERR_INVALID_ARG / VRT_ERR_RANGE as for the captured calls,
 * VRT_ERR_HIP if capture or instantiation fails. */
typedef struct vrt_graph vrt_graph;
vrt_status vrt_graph_create(vrt_ctx *ctx, const vrt_lines *lines, const vrt_grid *grid, const vrt_view *views,
                            const vrt_camera *cams, const vrt_image *imgs, int32_t n_passes, vrt_graph **out);
vrt_status vrt_graph_launch(vrt_graph *g, void *stream);
vrt_status vrt_graph_destroy(vrt_graph *g);

/* One frame without allocation, for callers that cannot allocate device memory
 * (work under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same kernels as vrt_voxelize(lines, grid), vrt_cull(view)
 * and vrt_trace(cam, img) in sequence, with no context.  The acceleration
 * structure lives in one fixed device array of VRT_NOALLOC_SCRATCH_BYTES per
 * device, which the library holds from the first call on that device until
 * the process ends; the call itself allocates nothing (no hipMalloc, no
 * allocating library routine).  The caller passes the inputs and the output
 * image, as for the per-stage calls (device pointers, borrowed until the
 * stream work completes).
 * Limits: n_vertices <= VRT_NOALLOC_MAX_VERTICES, every grid dimension <=
 * VRT_NOALLOC_MAX_DIM and width * height <= VRT_NOALLOC_MAX_PIXELS, else
 * VRT_ERR_CAPACITY before anything is enqueued; more than
 * VRT_NOALLOC_MAX_FRAGMENTS listed fragments latch VRT_ERR_CAPACITY on the
 * device.  Other argument errors as for the per-stage calls, also before
 * anything is enqueued.
 * info: NULL (nothing synchronizes; device errors of this frame are then not
 * reported) or filled as by vrt_frame_status (synchronizes the stream).
 * Every call on one device shares that device's array and the host state of
 * its frame, which keep the last call's contents (each call clears what it
 * needs at zero): calls that overlap on one device -- two streams, or two
 * threads -- race and must be serialized by the caller. */
#define VRT_NOALLOC_MAX_VERTICES 65536
#define VRT_NOALLOC_MAX_FRAGMENTS (1 << 20)
#define VRT_NOALLOC_MAX_DIM 64
#define VRT_NOALLOC_MAX_PIXELS (512 * 512)
#define VRT_NOALLOC_SCRATCH_BYTES (32 << 20)
vrt_status vrt_frame_noalloc(const vrt_lines *lines, const vrt_grid *grid, const vrt_view *view,
                             const vrt_camera *cam, const vrt_image *img, vrt_frame_info *info, void *stream);

/* Batched form: many independent line sets, each with its own grid, view,
 * camera and image, built and traced together.  VRT_BATCH_PERSISTENT runs
 * every stage of every set in ONE cooperative launch: the frame's stages are
 * phases separated by grid barriers, and inside a phase the resident blocks
 * take (set, stage, block) work items from a counter, largest sets first.
 * VRT_BATCH_STAGED runs the same phases as one launch each (kernel boundaries
 * instead of grid barriers; each phase kernel is compiled for its own stages,
 * so it keeps their register budget).  VRT_BATCH_SPLIT runs the view-
 * independent build (ingest, bins, pass 1, pyramid, erosion) in one
 * cooperative launch and every view-dependent phase (culling, lists, trace)
 * as a launch of its own after it.  VRT_BATCH_SEQUENTIAL issues the plain
 * vrt_voxelize / vrt_cull / vrt_trace calls set after set (the reference the
 * batched forms are compared with).  All give identical results.  Set i uses the arenas of a context created
 * from descs[i] (reachable with vrt_batch_context for vrt_frame_status and
 * vrt_query_as); all sets share one device.  vrt_batch_run validates every set
 * on the host before anything is enqueued and never allocates. */
#define VRT_BATCH_PERSISTENT 0
#define VRT_BATCH_SEQUENTIAL 1
#define VRT_BATCH_STAGED 2
#define VRT_BATCH_SPLIT 3

typedef struct {
    vrt_lines lines;
    vrt_grid grid;
    vrt_view view;
    vrt_camera cam;
    vrt_image image;
} vrt_batch_item;

typedef struct vrt_batch vrt_batch;
vrt_status vrt_batch_create(const vrt_desc *descs, int32_t n, vrt_batch **out);
vrt_status vrt_batch_run(vrt_batch *b, const vrt_batch_item *items, int32_t n, int32_t mode, void *stream);
vrt_status vrt_batch_context(vrt_batch *b, int32_t i, vrt_ctx **ctx);
vrt_status vrt_batch_destroy(vrt_batch *b);

/* Launch shape of the tracer (one per trace mode and context).  Every point
 * gives identical images; only the time differs.
 *   march_threads  threads per block of the march phase: 128, 256 or 512
 *                  (a block covers 16 x march_threads/16 pixels);
 *   shade_group    lanes that share one ray in the shade phase: 8, 16 or 32;
 *   shade_batch    list entries per lane whose records are fetched together: 2 or 4;
 *   lane_keys      transparent hits a lane keeps per pass over a list (k): 4 or 8;
 *   shade_blocks   size of the shade launch in units of 256 threads: 256 .. 65535
 *                  (launched as single-wave workgroups, four per unit).
 * Default {256, 16, 2, 4, 4096}.  The persistent and staged batch forms use
 * each set's shade_group (its context's shape for the set's trace mode, e.g.
 * after vrt_autotune on vrt_batch_context) and the defaults for the rest. */
typedef struct {
    int32_t march_threads;
    int32_t shade_group;
    int32_t shade_batch;
    int32_t lane_keys;
    int32_t shade_blocks;
    int32_t reserved[3]; /* zero */
} vrt_tune;

/* Sets / reads the launch shape used by vrt_trace (and graphs captured
 * afterwards) for trace mode `mode`.  Errors: VRT_ERR_INVALID_ARG for a null
 * pointer, a bad mode or a value outside the sets above (nothing changes). */
vrt_status vrt_set_tune(vrt_ctx *ctx, int32_t mode, const vrt_tune *tune);
vrt_status vrt_get_tune(vrt_ctx *ctx, int32_t mode, vrt_tune *tune);

/* Host-timed search of the launch shape for the context's current
 * acceleration structure and one camera (its mode selects which shape is
 * tuned): coordinate descent from the current shape over the sets above, one
 * parameter at a time, for `sweeps` sweeps or until a sweep changes nothing.
 * Each point is traced `warmup` times untimed, then `reps` times between two
 * HIP events on `stream`; its time is the mean.  The best shape is set on
 * the context.  With a cache file, the result is looked up first under the
 * key "<gfx arch>|<form>|<mode>|<grid dims>|<W>x<H>|<n_vertices>|<key>" and
 * stored after a search (a JSON object, one entry per line, rewritten
 * through a temporary file).  Writes the image buffers; synchronizes.
 * Errors: as vrt_trace; VRT_ERR_INVALID_ARG for reps < 1, warmup < 0,
 * sweeps < 1; a cache file that cannot be read or written is ignored. */
typedef struct {
    const vrt_camera *cam;
    const vrt_image *image;  /* device buffers written by every timed trace */
    int32_t reps;
    int32_t warmup;
    int32_t sweeps;
    int32_t reserved;
    const char *cache_path;  /* NULL: no cache */
    const char *key;         /* caller's workload name (NULL: empty) */
} vrt_tune_space;

typedef struct {
    vrt_tune best;
    float best_ms;      /* mean trace time of the best shape */
    float start_ms;     /* mean trace time of the shape the search started from */
    int32_t evaluated;  /* shapes timed (0 on a cache hit) */
    int32_t from_cache; /* 1 when the shape came from the cache file */
} vrt_tune_result;

vrt_status vrt_autotune(vrt_ctx *ctx, const vrt_tune_space *space, vrt_tune_result *out, void *stream);

/* Host-timed choice of the grid resolution for one line set.  The grid only
 * narrows the search for hits (voxelization and culling are conservative), so
 * every grid yields the same hits up to binary32 rounding of the hit
 * parameters; fragment counts, list lengths and walk lengths change with it.
 * For each of the n_grids candidates: one frame (vrt_voxelize, then vrt_cull
 * and vrt_trace for each of the n_passes (view, camera, image) triples),
 * vrt_frame_status, `warmup` untimed frames and `reps` frames between two HIP
 * events on `stream`.  ms[i] (host, n_grids entries) receives the mean frame
 * time, or +inf when the candidate latched a device error (e.g. it needs
 * more than max_fragments); *best the index of the fastest.  The context
 * holds the last candidate's structure afterwards.  Writes the image buffers;
 * synchronizes.  Errors: VRT_ERR_INVALID_ARG (null pointers, counts < 1,
 * warmup < 0), any error of the frame's calls (e.g. an invalid grid), or the
 * device error of the last candidate when none fits. */
vrt_status vrt_autotune_grid(vrt_ctx *ctx, const vrt_lines *lines, const vrt_grid *grids, int32_t n_grids,
                             const vrt_view *views, const vrt_camera *cams, const vrt_image *imgs, int32_t n_passes,
                             int32_t reps, int32_t warmup, int32_t *best, float *ms, void *stream);

/* Synchronizes the context's last stream, reads the device status word and
 * the frame totals, and clears the latched error. */
vrt_status vrt_frame_status(vrt_ctx *ctx, vrt_frame_info *out);

/* Fills device pointers to the acceleration structure (synchronizes to read
 * the brick count). */
vrt_status vrt_query_as(vrt_ctx *ctx, vrt_as_view *out);

/* Writes the binary32 primary-ray directions of n pixels (indices y*W + x)
 * into dirs[3*n] (device) -- the exact rays vrt_trace uses. */
vrt_status vrt_debug_rays(vrt_ctx *ctx, const vrt_camera *cam, const int64_t *pixels, int64_t n, float *dirs,
                          void *stream);

/* Per-kernel timing: when enabled, every kernel the context launches is
 * bracketed by a pair of HIP events recorded on its launch stream (up to
 * 65536 launches between reads).  vrt_profile_read synchronizes, writes one
 * record per kernel name (launch count and summed event time), and resets. */
typedef struct {
    char name[32];
    int64_t launches;
    double total_ms;
} vrt_kernel_time;

vrt_status vrt_profile_enable(vrt_ctx *ctx, int32_t enable);
vrt_status vrt_profile_read(vrt_ctx *ctx, vrt_kernel_time *out, int32_t max_records, int32_t *n_records);

/* Work counters of one trace (inspection): the same trace as vrt_trace, run
 * with per-ray counters and marks of the voxels and segments it touches;
 * writes the image too.  Synchronizes. */
typedef struct {
    int64_t rays;               /* W * H */
    int64_t rays_hit;           /* rays with a first hit */
    int64_t cell_skips_64;      /* empty 64^3 cells crossed in one step */
    int64_t cell_skips_8;       /* invisible bricks, 16^3 and 32^3 cells crossed in one step */
    int64_t voxel_steps;        /* voxels visited in non-empty bricks */
    int64_t list_visits;        /* visits of voxels with a non-empty list */
    int64_t capsule_tests;      /* ray-capsule tests, repeats included */
    int64_t kbuffer_passes;     /* transparent: passes over a voxel list */
    int64_t distinct_list_voxels;  /* voxels whose list was read by any ray */
    int64_t distinct_list_entries; /* sum of the list lengths of those voxels */
    int64_t distinct_segments;     /* segments tested by any ray */
    int64_t max_tests_per_ray;
} vrt_trace_stats;

vrt_status vrt_trace_stats_run(vrt_ctx *ctx, const vrt_camera *cam, const vrt_image *out, vrt_trace_stats *stats,
                               void *stream);

/* Memory-system ceilings the frame's kernels are measured against (one
 * launch between two HIP events on `stream`; synchronizes; *ms its time):
 *   VRT_MB_COPY           copies the first half of buf (device, `bytes`) to
 *                         the second half (`bytes` moved in total; ops unused);
 *   VRT_MB_ATOMIC_RANDOM  `ops` 32-bit atomic adds of 1 on pseudo-random words
 *                         of buf (the per-fragment atomics of voxelization
 *                         pass 1, Section 3.1, at no locality);
 *   VRT_MB_ATOMIC_BRICK   `ops` such adds where the 64 of one wave step fall in
 *                         one 2 KiB region (one brick's packed words).
 * buf's contents are overwritten.  Errors: VRT_ERR_INVALID_ARG (null pointer,
 * bytes not a positive multiple of 4096, ops < 1 for the atomics, bad kind),
 * VRT_ERR_HIP. */
#define VRT_MB_COPY 0
#define VRT_MB_ATOMIC_RANDOM 1
#define VRT_MB_ATOMIC_BRICK 2
vrt_status vrt_microbench(int32_t kind, void *buf, int64_t bytes, int64_t ops, float *ms, void *stream);

/* Synchronous copy of `bytes` from device memory to host memory. */
vrt_status vrt_copy_to_host(void *host_dst, const void *device_src, int64_t bytes);

/* The HIP error code of the last VRT_ERR_HIP on this thread. */
int32_t vrt_last_hip_error(void);

/* Static description of a status code. */
const char *vrt_status_string(vrt_status s);

#ifdef __cplusplus
}
#endif

#endif /* VRT_H */
