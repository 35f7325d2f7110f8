/*
 * shadow_accrual.h -- C ABI of the MI355X (gfx950) shadow-accumulation
 * library (libsa).
 *
 * What it computes: for every sample point of a city (ground or facade),
 * the time it spends in the shadow of extruded buildings over a time span
 * -- the paper's "gross shadow" (Sec. 3.1) -- in two forms:
 *
 *   SA_SAMPLED  one shadow ray per point per sun instant, the per-step
 *               ray-casting approach the paper uses as its baseline
 *               (Sec. 8.1, "brute force ray tracing");
 *   SA_ACCRUAL  the sun-movement form: between two knot instants the light
 *               direction turns along a great circle at a constant angular
 *               rate (the motion under which Theorem 1 of Sec. 4 holds), so
 *               the rays from a point sweep a planar fan and every occluder
 *               contributes one occluded time interval (the shadow of each
 *               source moves along a line, Sec. 3.2; all sources are taken,
 *               Sec. 5); the union of those intervals is measured.
 *
 * Frame: local east-north-up metres (x east, y north, z up), ground z = 0.
 * Buildings are convex prisms: a counter-clockwise convex footprint
 * extruded from z = 0 to z = H > 0, closed.  The sun is a directional
 * light (Sec. 3.2).
 *
 * Conventions:
 *  - Every call returns sa_status; 0 is success, negative an error.  No
 *    call aborts or throws; the context keeps a message (sa_last_error).
 *  - Device work is enqueued on the context's HIP stream; calls return
 *    after enqueueing.  The only host-synchronous calls are the ones that
 *    build library-owned objects (scene upload / height edit, path
 *    upload) and sa_sync.
 *  - "host" pointers are read before the call returns and may be freed
 *    after; "device" pointers are caller-owned device memory (e.g. torch
 *    tensors), never freed by the library and read or written by work on
 *    the context's stream.
 *  - Scenes and paths are library-owned, opaque, freed by their destroy
 *    call.  All objects belong to the context that made them.
 */
#ifndef SHADOW_ACCRUAL_H
#define SHADOW_ACCRUAL_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t sa_status;
#define SA_OK 0
#define SA_ERR_INVALID_ARG (-1)  /* bad pointer, size, mode or range */
#define SA_ERR_GEOMETRY (-2)     /* footprint not convex / not CCW / < 3 vertices, H <= 0 */
#define SA_ERR_CAPACITY (-3)     /* a fixed-size structure overflowed (BVH depth, spill queue) */
#define SA_ERR_OOM (-4)          /* device allocation failed */
#define SA_ERR_DEVICE (-5)       /* HIP runtime error */
#define SA_ERR_UNSUPPORTED (-6)  /* a request the library does not handle */

#define SA_SAMPLED 0
#define SA_ACCRUAL 1

/* sa_accum_opts.flags */
#define SA_FLAG_ADD 1u           /* add into the outputs instead of overwriting them */

typedef struct sa_ctx sa_ctx;
typedef struct sa_scene sa_scene;
typedef struct sa_path sa_path;

/* ------------------------------------------------------------------ */
/* context                                                             */
/* ------------------------------------------------------------------ */

/* Create a context on HIP device `device`, enqueueing on `hip_stream`
 * (a hipStream_t; NULL = the default stream). */
sa_status sa_create(int32_t device, void *hip_stream, sa_ctx **out);
void sa_destroy(sa_ctx *ctx);
/* Change the stream later calls enqueue on. */
sa_status sa_set_stream(sa_ctx *ctx, void *hip_stream);

/* Launch choices of a context that change speed, never results (counts and
 * bit vectors are equal under every choice; minutes may differ in the last
 * bits where a bin's float sums are grouped differently).  An autotuner
 * measures them per device and sets them; zero fields keep the defaults. */
typedef struct {
    int32_t accrual_segments_per_launch; /* accrual form: the most path segments one launch covers
                                            (their per-segment hierarchy views are the launch's working
                                            set); 0 = as many as the view budget allows */
    int32_t batched_grid_blocks;         /* sa_accumulate_batched: blocks of the persistent launch when
                                            opts->grid_blocks is 0; 0 = 2048 */
    int32_t batched_tiles_per_grab;      /* sa_accumulate_batched: consecutive 64-point tiles a wave takes
                                            from the work queue per atomic; 0 = 1 */
    int32_t tile_grid_blocks;            /* sa_accumulate (both forms) and sa_building_contribution:
                                            blocks (of 256 threads) of their persistent launches, whose
                                            waves take (64-point tile, bin) units from a work counter
                                            per XCD; 0 = as many as the device holds at once */
    int32_t accrual_waves_per_simd;      /* accrual form: occupancy variant of its kernel, 6, 7 or 8
                                            waves per SIMD (registers per lane shrink as it grows);
                                            0 = 8 */
    int32_t sampled_instants_per_packet; /* sampled form: instants a wave's packet takes per point,
                                            1, 2, 4, 8 or 16 (so 64 down to 4 points); 0 = 8 */
    int32_t reserved[2];                 /* 0 */
} sa_launch;
/* Errors: INVALID_ARG (negative or out-of-range values). */
sa_status sa_set_launch(sa_ctx *ctx, const sa_launch *launch);
sa_status sa_get_launch(const sa_ctx *ctx, sa_launch *out);
/* Message of the last failed call on this context ("" if none). */
const char *sa_last_error(const sa_ctx *ctx);
/* Wait for the context's stream; reports errors raised by device work
 * since the last sync and clears them: CAPACITY if the accrual spill queue
 * overflowed or an occluded set could not be split finely enough (results
 * incomplete), INVALID_ARG if a batched variant named a bad building id or
 * height. */
sa_status sa_sync(sa_ctx *ctx);
/* Library version string. */
const char *sa_version(void);
/* Measurement aid for the roofline, not a step of the method: the vector
 * ALU's FP32 lane-op rate on the context's device, measured with chains of
 * independent fused multiply-adds (one VALU operation per lane each) on the
 * context's stream; the best of three timed launches after a warm-up.
 * Host-synchronous; allocates nothing (its never-taken store points into
 * the context's own queue).  *lane_ops_per_s: host double.  Errors:
 * INVALID_ARG, DEVICE. */
sa_status sa_measure_valu_peak(sa_ctx *ctx, double *lane_ops_per_s);

/* ------------------------------------------------------------------ */
/* scene: buildings as extruded convex prisms (a city model, Sec. 8.2) */
/* ------------------------------------------------------------------ */

/* Upload n_b prisms from arrays vert_off [n_b+1] (CSR offsets into xy),
 * xy [2*vert_off[n_b]] (x, y pairs, counter-clockwise, convex, >= 3
 * vertices), height [n_b] (> 0).  Each array may be host or device memory
 * (told apart by the runtime's pointer attributes; device arrays are read
 * through a host copy for validation); all are copied in, the caller keeps
 * ownership.  Builds the bounding-volume hierarchy on
 * the device (Morton codes of footprint centres, radix sort, binary radix
 * tree, bottom-up box refit).  Host-synchronous.  n_b == 0 is an empty
 * scene (nothing casts shadow); at most 2^25 prisms.  Errors: INVALID_ARG,
 * GEOMETRY, CAPACITY (more than 2^25 prisms, or a tree deeper than 64
 * levels), OOM, DEVICE. */
sa_status sa_scene_upload(sa_ctx *ctx, int32_t n_b, const int32_t *vert_off,
                          const float *xy, const float *height, sa_scene **out);

/* Replace the heights of buildings ids[0..n) (original building ids) by
 * h[0..n) (> 0) and refit the hierarchy's boxes (heights only: the
 * topology is kept).  Models the paper's impact analysis, where a building
 * is replaced and the shadows recomputed (Sec. 7.1).  Host arrays: checked
 * on the host (INVALID_ARG / GEOMETRY), host-synchronous.  Device arrays
 * (both; e.g. the heights a gradient step produced): written and refitted
 * on the context's stream with no host round trip; an id out of range or a
 * height that is not a positive finite number is skipped and reported by
 * the next sa_sync (INVALID_ARG). */
sa_status sa_scene_set_heights(sa_ctx *ctx, sa_scene *scene, int32_t n, const int32_t *ids,
                               const float *h);

typedef struct {
    int32_t n_b;      /* prisms */
    int32_t n_vert;   /* footprint vertices */
    int32_t n_nodes;  /* interior hierarchy nodes (n_b - 1, or 1 if n_b == 1) */
    int32_t depth;    /* levels from the root to the deepest leaf */
    float bounds[4];  /* xmin, ymin, xmax, ymax of the footprints */
    float max_height;
} sa_scene_info;
sa_status sa_scene_get_info(const sa_scene *scene, sa_scene_info *out);

/* Copy the hierarchy to the host for inspection: nodes [n_nodes * 16]
 * 32-bit words (layout in the library source: per interior node the two
 * child boxes and child references) and prim_order [n_b] (original id of
 * the prism at each leaf position).  Either pointer may be NULL. */
sa_status sa_scene_read_bvh(sa_ctx *ctx, const sa_scene *scene, void *nodes, int32_t *prim_order);

void sa_scene_destroy(sa_scene *scene);

/* ------------------------------------------------------------------ */
/* sun path: the time selection of Sec. 7.1 (start date, n days, a      */
/* daily window) turned into sample instants and great-circle knots      */
/* ------------------------------------------------------------------ */

typedef struct {
    double lat_deg, lon_deg;  /* site, degrees (east positive) */
    double tz_offset_h;       /* local civil time = UTC + tz_offset_h */
} sa_site;

typedef struct {
    int32_t year, month, day; /* first day (Gregorian) */
    int32_t n_days;           /* consecutive days, >= 1 */
    double t_start_min;       /* local minutes after midnight; < 0: the first whole minute
                                 with the sun above the horizon */
    double t_end_min;         /* with t_start_min < 0: ignored (last such minute) */
    double step_min;          /* spacing of the sample instants (> 0) */
    double seg_min;           /* knot spacing of the accrual form (> 0) */
    int32_t knot_clock;       /* 0: knots at t0, t0 + seg_min, ..., and t1 (t0, t1: the day's
                                 first and last instants); 1: at t0, at every multiple of
                                 seg_min in local time inside (t0, t1), and at t1, so that
                                 different days share knot times (the direction graph then
                                 merges more of their segments) */
} sa_timespan;

/* Host arrays describing a sun path.  As the output of sa_sunpath the
 * caller sets the cap_* fields and the array pointers (or NULL to only
 * size); as the input of sa_path_upload all counts and arrays are read. */
typedef struct {
    int32_t n_days, n_samples, n_knots;
    int32_t cap_days, cap_samples, cap_knots;
    int32_t *day_sample_off; /* [n_days+1] samples of day d: [off[d], off[d+1]) */
    double *t_min;           /* [n_samples] local minutes of each instant */
    double *dir;             /* [3*n_samples] unit direction toward the sun (E, N, U) */
    double *weight;          /* [n_samples] minutes each instant stands for (its share of
                                the day's span; ends get half a step) */
    int32_t *day_knot_off;   /* [n_days+1] knots of day d: [off[d], off[d+1]) */
    double *knot_t;          /* [n_knots] knot instants (local minutes): the span start,
                                every seg_min after it, and the span end */
    double *knot_dir;        /* [3*n_knots] */
    int32_t *day_bin;        /* [n_days] output bin of each day; NULL on input = bin = day */
} sa_sunpath_buf;

/* Solar position by the NOAA solar-calculator equations (Meeus' low
 * precision solar coordinates), geometric elevation (no refraction), FP64.
 * Fills `out` for the days of `span`; days keep only instants with the sun
 * above the horizon (a fixed window that reaches below it is an
 * INVALID_ARG).  Sizing: with cap_* == 0 only the counts are written.
 * Host only, synchronous.  Errors: INVALID_ARG, CAPACITY (caps too small). */
sa_status sa_sunpath(const sa_site *site, const sa_timespan *span, sa_sunpath_buf *out);

/* Upload a sun path (host arrays of `in`, any number of days, each day's
 * knots spanning its samples) for use by accumulate calls.  Precomputes,
 * in FP64 on the host, each segment's plane, basis and angle.  Bins:
 * in->day_bin (or bin = day); n_bins = 1 + max bin.  Errors: INVALID_ARG,
 * OOM. */
sa_status sa_path_upload(sa_ctx *ctx, const sa_sunpath_buf *in, sa_path **out);

/* As sa_path_upload, with the direction graph of Sec. 6 for the accrual
 * form: the hemisphere is cut into cells of about bound_deg (rings of
 * that height in elevation, each cut into the fewest equal azimuth sectors
 * no wider than bound_deg at the ring's lower edge), and segments of one
 * output bin whose start and end knots fall in the same pair of cells
 * become one edge, computed once on the members' mean arc (the normalised
 * mean of their start directions to that of their end directions) and
 * weighted by their number (Eq. (1)).  Each merged segment keeps its own
 * duration; sample counts are the edge's times its multiplicity.  Every
 * accrual-form call takes the graph: sa_accumulate, sa_accumulate_batched,
 * sa_building_contribution and sa_grad_heights.  An approximation for long
 * spans: each member's arc lies up to about bound_deg from the edge's, and
 * the offsets cancel to first order in the summed minutes (a year in season
 * bins: 0.34 minutes per point and day at 3 degrees).  The sampled form
 * is unaffected; the continuous shadow needs time order and is refused
 * (INVALID_ARG).  bound_deg in [1e-6, 90].  Errors as sa_path_upload. */
sa_status sa_path_upload_graph(sa_ctx *ctx, const sa_sunpath_buf *in, double bound_deg, sa_path **out);
sa_status sa_path_info(const sa_path *path, int32_t *n_bins, int32_t *n_samples,
                       int32_t *n_segments);
void sa_path_destroy(sa_path *path);

/* ------------------------------------------------------------------ */
/* accumulate: gross shadow per point (Sec. 3.1), binned by day          */
/* ------------------------------------------------------------------ */

/* Sample points, device arrays of n float32 (structure of arrays).
 * Ground points: z = 0, nx = ny = 0, owner = -1.  Facade points: on a wall
 * of building `owner` (original id), (nx, ny) the wall's outward
 * horizontal normal; a wall facing away from the sun is in shadow.  nx, ny,
 * owner may be NULL (all ground / no owner). */
typedef struct {
    int64_t n;
    const float *x, *y, *z;
    const float *nx, *ny;
    const int32_t *owner;
} sa_points;

typedef struct {
    int32_t mode;     /* SA_SAMPLED or SA_ACCRUAL */
    uint32_t flags;   /* SA_FLAG_ADD */
    float out_scale;  /* minutes are multiplied by this (0 = 1; 1/60 gives hours) */
    int32_t grid_blocks; /* sa_accumulate_batched: blocks of 256 threads in the persistent
                            launch (0 = default 2048); ignored elsewhere */
    /* Optional device uint64 [8], added to (not cleared): when non-NULL the
     * launch runs an instrumented instantiation that counts, per lane, the
     * work its own traversal needed -- [0] child-box tests, [1] prism tests,
     * [2] footprint edges visited in prism tests, [3] interval insertions,
     * [4] node fetches (per wave), [5] lanes x units (point-instants or
     * point-segments), [6] spilled windows, [7] leaf visits (per wave).  Slower; for
     * measurement only. */
    uint64_t *work;
    /* Optional device float [n_bins * n] (bin-major; NULL = not wanted):
     * continuous shadow (Sec. 3.1) -- the longest time the point stays in
     * shadow without interruption within one day, in minutes times
     * out_scale, the maximum over the bin's days.  SA_SAMPLED: the longest
     * run of consecutive shadowed instants (Sec. 5), as the sum of their
     * weights; SA_ACCRUAL: the longest member of the day's shadowed set
     * along the path, runs that meet at a knot being one run (Sec. 6 joins
     * per-segment prefix / longest / suffix the same way).  Cleared first
     * unless SA_FLAG_ADD, which keeps the larger of the stored and the new
     * value.  With it the accrual form resolves sets of more than four
     * pieces in segment order inside the kernel (slower).
     * sa_accumulate_batched: must be NULL. */
    float *longest;
    /* Optional device double [n_bins * n] (bin-major; NULL = not wanted;
     * SA_ACCRUAL only, not sa_accumulate_batched): the accrual minutes
     * before their rounding to float32 -- each lane sums its segment
     * measures in FP64 -- times out_scale, e.g. for loss totals whose
     * differences must not carry float32 rounding.  Cleared first unless
     * SA_FLAG_ADD. */
    double *minutes64;
} sa_accum_opts;

/* Gross shadow of every point over every day of `path`, summed per bin.
 *   counts  device int32 [n_bins * n] (bin-major; NULL = not wanted):
 *           SA_SAMPLED: shadowed instants; SA_ACCRUAL: sample instants
 *           inside the occluded set.
 *   minutes device float [n_bins * n]: SA_SAMPLED: sum of the weights of the
 *           shadowed instants; SA_ACCRUAL: measure of the occluded set (both
 *           times out_scale).
 *   bits    device uint32 [ceil(n_samples/32) * n] (word-major; SA_SAMPLED
 *           only; NULL = not wanted): bit k%32 of word k/32 of point i is
 *           instant k's predicate -- the n-bit shadow vector of Sec. 5.
 * Results are deterministic except in the last bits of minutes for points
 * with a spilled point-segment (more than four pieces), whose measures are
 * added with float atomics in no fixed order.
 * The accrual form (here, and in sa_accumulate_batched, sa_grad_heights
 * and sa_building_contribution) keeps a per-segment view of the hierarchy
 * (64 bytes per node and segment, at most 256 MiB per launch; longer paths
 * run as several launches, the continuous shadow one day at least) in
 * memory the context owns: grown on first need with the stream
 * synchronised, kept until sa_destroy.  Under stream capture make one
 * eager call of the same (or a larger) size first.
 * Errors: INVALID_ARG, CAPACITY (reported by sa_sync if the accrual spill
 * queue overflows), OOM, DEVICE. */
sa_status sa_accumulate(sa_ctx *ctx, const sa_scene *scene, const sa_points *pts,
                        const sa_path *path, const sa_accum_opts *opts, int32_t *counts,
                        float *minutes, uint32_t *bits);

/* For callers that cannot allocate device memory during a call (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation): sa_accumulate with the same arguments, outputs and results,
 * except that it allocates nothing.  The accrual form's per-segment
 * hierarchy views (64 bytes per node and segment) go to a fixed device
 * array of SA_NOALLOC_SCRATCH_BYTES that every device the library runs on
 * holds from its first sa_create until the process ends, and the spill
 * queue is the one sa_create made for the context; the sampled form needs
 * no scratch.  A launch covers as many segments as the array holds
 * (SA_NOALLOC_SCRATCH_BYTES / (64 x interior nodes): 52 on a 20,000-prism
 * scene), longer paths run as several launches; with opts->longest a
 * launch must hold a whole day.  Every call on one device shares the array
 * and its contents are rebuilt by each launch, so calls that overlap on one
 * device (other streams or contexts) race and must be ordered by the
 * caller.  Errors: as sa_accumulate; CAPACITY (before any work is
 * enqueued) when one segment's views (a scene of more than about 1M
 * prisms) or, with longest, one day's views exceed the array; DEVICE if the
 * array's address could not be obtained at sa_create. */
#define SA_NOALLOC_SCRATCH_BYTES (64ll << 20)
sa_status sa_accumulate_noalloc(sa_ctx *ctx, const sa_scene *scene, const sa_points *pts,
                                const sa_path *path, const sa_accum_opts *opts, int32_t *counts,
                                float *minutes, uint32_t *bits);

/* Batched development scenarios (Sec. 7.1 impact analysis, many at once):
 * n_var variants of `scene`, variant v replacing the heights of buildings
 * var_ids[v*k .. v*k+k) by var_h[v*k ..) (device arrays, original ids,
 * k = ids_per_var), each evaluated on its own points
 * pts[var_off[v] .. var_off[v+1]) (var_off: device int64 [n_var+1]).  One
 * refit per variant and one persistent accrual launch over a (variant,
 * tile) work queue.  Outputs as sa_accumulate over the concatenated points
 * (SA_ACCRUAL only). */
sa_status sa_accumulate_batched(sa_ctx *ctx, const sa_scene *scene, int32_t n_var,
                                int32_t ids_per_var, const int32_t *var_ids, const float *var_h,
                                const sa_points *pts, const int64_t *var_off,
                                const sa_path *path, const sa_accum_opts *opts, int32_t *counts,
                                float *minutes);

/* Gradient of L = sum_bins sum_p dl_dmin[bin*n + p] * minutes_accrual(p, bin)
 * (minutes times opts->out_scale) with respect to every building height:
 * each boundary of a point's occluded set that is made by a roof edge
 * moves with the height; its time derivative comes from implicit
 * differentiation of the roof-grazing condition (closing ends +, opening
 * ends -).  Traversals are recomputed, nothing is stored from the forward
 * pass; contributions are summed per building across each wave and
 * accumulated in FP64, then rounded once.  opts: NULL or mode SA_ACCRUAL
 * (the sampled form's counts are piecewise constant in the heights);
 * out_scale and SA_FLAG_ADD (add into grad instead of overwriting it) are
 * honoured, the other fields ignored.  dl_dmin: device float [n_bins * n]
 * or NULL (all ones).  grad: device float [n_b] (original ids).
 * Errors: INVALID_ARG, OOM, DEVICE. */
sa_status sa_grad_heights(sa_ctx *ctx, const sa_scene *scene, const sa_points *pts,
                          const sa_path *path, const sa_accum_opts *opts, const float *dl_dmin,
                          float *grad);

/* Building contribution (Sec. 7.2): per output bin and building, the time
 * the points spend in that building's own shadow along the great-circle
 * path of `path` (the accrual form), weighted per point (e.g. by the area a
 * point stands for).  A moment shadowed by several buildings counts for
 * each of them; a facade point's wall facing away from the sun counts for
 * its own building; a point under a roof counts its whole span for that
 * building.
 *   weight   device float [n] or NULL (all ones)
 *   contrib  device double [n_bins * n_b], bin-major, original building ids;
 *            overwritten (minutes x weight).
 * Errors: INVALID_ARG, DEVICE. */
sa_status sa_building_contribution(sa_ctx *ctx, const sa_scene *scene, const sa_points *pts,
                                   const sa_path *path, const float *weight, double *contrib);

typedef struct {
    float texel_m;       /* texel edge on the shadow plane, metres (> 0) */
    float bias_m;        /* depth margin of the shadow test, metres (>= 0) */
    float box[6];        /* x0, y0, z0, x1, y1, z1: a box that holds every prism; all zero =
                            the footprints' extent, 0 .. the tallest height the scene has had */
    uint32_t flags;      /* SA_FLAG_ADD */
    float out_scale;     /* minutes are multiplied by this (0 = 1) */
    int64_t max_texels;  /* cap on one segment's map, slices x texels (0 = 2^31) */
} sa_sam_opts;

/* Gross shadow by raster shadow accrual maps (Sec. 4), the exploration
 * form: per path segment one map with a depth slice per sample instant
 * (the instant's direction on the great circle between the knots, as in
 * the accrual form), over a grid of texel_m squares on a plane normal to
 * the segment's start direction, 1 m behind the box corner farthest from
 * the sun.  Step 1 fills every slice in one pass over (slice, prism) pairs:
 * a texel holds the largest distance along the light at which the ray from
 * its centre toward the sun leaves a prism.  Step 2 puts each point's
 * shadow on every slice and counts the instants whose stored depth exceeds
 * the point's own by more than bias_m.  A raster approximation of
 * sa_accumulate's sampled form, exact as texel_m -> 0 away from shadow
 * edges; prisms outside `box` are missed.  Points: ground-type only (any
 * z; pts->owner, nx and ny must be NULL: walls would shade themselves).
 * Outputs as sa_accumulate (counts int32, minutes float, [n_bins * n],
 * either may be NULL).  The library keeps one segment's map (4 bytes per
 * texel and slice: a segment stamp and the depth to about 1 / 2^24 of its
 * range) in memory the context owns, grown on first need; calls on one
 * context must not overlap.  Not
 * for direction-graph paths.
 * Errors: INVALID_ARG, CAPACITY (a map above max_texels), OOM, DEVICE. */
sa_status sa_sam_accumulate(sa_ctx *ctx, const sa_scene *scene, const sa_points *pts,
                            const sa_path *path, const sa_sam_opts *opts, int32_t *counts,
                            float *minutes);

/* Daylight minutes of every output bin of a path: the sum of its days'
 * spans.  span: host double [n_bins].  Errors: INVALID_ARG. */
sa_status sa_path_bin_span(const sa_path *path, double *span);

/* Region shadow score (Sec. 7.2): out[r] = sum over p in
 * [region_off[r], region_off[r+1]) of (area ? area[p] : 1) times
 * sum over the path's bins b of interval_weight[b] * values[b * n + p] /
 * span_b, accumulated in FP64, with span_b the bin's daylight minutes (the
 * sum of its days' spans, as sa_path_bin_span gives).  With values = the
 * per-bin shadow minutes of `path` and interval_weight[b] in [-1, 1] the
 * interval's weight, this is the score: the weighted fraction of each
 * interval's daylight spent in shadow, summed over the region.
 * values: device float [n_bins * n] (bin-major, n_bins = the path's);
 * interval_weight: host double [n_bins], read before the call returns;
 * region_off: device int64 [n_reg+1]; area: device float [n] or NULL;
 * out: device double [n_reg].  Host-synchronous (the per-bin weights are
 * uploaded).  Errors: INVALID_ARG (also a bin without daylight), OOM,
 * DEVICE. */
sa_status sa_region_score(sa_ctx *ctx, const sa_path *path, const float *values, int64_t n,
                          const double *interval_weight, const int64_t *region_off, int32_t n_reg,
                          const float *area, double *out);

/* Region sums (the shadow area of Sec. 7.2): out[r] = sum over
 * p in [region_off[r], region_off[r+1]) of values[p] * (area ? area[p] : 1),
 * accumulated in FP64.  values, area: device float [n]; region_off: device
 * int64 [n_reg+1]; out: device double [n_reg]. */
sa_status sa_region_sum(sa_ctx *ctx, const float *values, int64_t n, const int64_t *region_off,
                        int32_t n_reg, const float *area, double *out);

#ifdef __cplusplus
}
#endif
#endif /* SHADOW_ACCRUAL_H */
