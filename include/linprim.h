/*
 * linprim.h -- C ABI of the MI355X (gfx950) differentiable tile rasterizer
 * for transparent linear primitives: octahedra and tetrahedra, following
 * LinPrim (von Luetzow & Niessner, arXiv 2501.16312).
 *
 * Pipeline (Sec. 3.2 "Rendering Process", Sec. 3.4 "Optimization"):
 *   linprim_preprocess  -> per primitive and view: build the primitive from
 *                          its features, transform it to the camera, colour
 *                          it from its SH along the viewing direction,
 *                          project it into the EWA affine ray space and bound
 *                          it on screen; count the tiles it touches and
 *                          prefix-sum the counts.
 *   linprim_bin_sort    -> one (tile | depth, primitive) pair per touched
 *                          tile, sorted by key ("Global Sorting and Tiling"),
 *                          and the [start, end) range of every tile.
 *   linprim_render_fwd  -> per pixel, front-to-back compositing of the tile's
 *                          list with the chord-based opacity of Eq. 1 and
 *                          App. E, stopping once cumulative opacity reaches
 *                          0.999 ("Rasterization", "Compositing").
 *   linprim_render_bwd  -> gradients of a loss given dL/dC, through blending,
 *                          chords, ray space and the view transform down to
 *                          the primitive features ("Rasterization/
 *                          Preprocessing Backpropagation", App. E).
 *
 * Conventions shared by every entry point:
 *   - Every array argument is a DEVICE pointer owned by the caller, except
 *     the linprim_camera array, the background colour and the outputs of
 *     linprim_pair_count / linprim_read_status, which are HOST pointers.
 *   - Calls only enqueue work on `stream` (a hipStream_t; NULL = the null
 *     stream) and return at once; none allocates device memory.  The single
 *     call that waits for the stream is linprim_pair_count (it must return a
 *     number to the host).
 *   - Return value: LINPRIM_OK (0) or a negative LINPRIM_ERR_* code; the
 *     outputs are then untouched.  linprim_strerror names the code.
 *   - Degenerate primitives (zero quaternion, a distance <= 0, non-finite
 *     values, opacity outside [0, 1], centre not beyond the near plane, or a
 *     box that covers no pixel centre) are culled, not reported.
 */
#ifndef LINPRIM_H
#define LINPRIM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { LINPRIM_OCTAHEDRON = 0, LINPRIM_TETRAHEDRON = 1 };

enum {
    LINPRIM_OK = 0,
    LINPRIM_ERR_INVALID_ARG = -1,     /* null pointer, bad size, unknown type or tile */
    LINPRIM_ERR_WORKSPACE = -2,       /* a workspace is smaller than its *_size() */
    LINPRIM_ERR_PAIR_OVERFLOW = -3,   /* more (tile, primitive) pairs than max_pairs */
    LINPRIM_ERR_HIP = -4,             /* a HIP launch or query failed */
    LINPRIM_ERR_DEVICE = -5           /* current device is not gfx950 */
};

/* Primitives (Sec. 3.1).  Octahedron: centre mu, rotation q, one distance per
 * pair of opposite vertices (corners mu +/- R(q) d_k e_k).  Tetrahedron:
 * centre mu, rotation q, one distance per corner along four equally spaced
 * directions (corners mu + R(q) d_i b_i, b_i = (1,1,1), (1,-1,-1), (-1,1,-1),
 * (-1,-1,1) over sqrt(3)).  All float32, row-major, device memory. */
typedef struct linprim_prims {
    int32_t type;          /* LINPRIM_OCTAHEDRON or LINPRIM_TETRAHEDRON */
    int32_t sh_degree;     /* 0..3: (sh_degree+1)^2 coefficients per channel */
    int64_t n;             /* number of primitives, 0 <= n < 2^31 */
    const float *means;    /* [n,3] */
    const float *quats;    /* [n,4] (w,x,y,z); need not be unit, normalised inside */
    const float *dists;    /* [n,3] octahedron, [n,4] tetrahedron; > 0 */
    const float *opacity;  /* [n] activated opacity alpha in [0,1] (Eq. 1) */
    const float *sh;       /* [n,(sh_degree+1)^2,3] SH coefficients, RGB last */
} linprim_prims;

/* Pinhole camera, OpenCV axes (x right, y down, z forward).  HOST struct. */
typedef struct linprim_camera {
    float world_to_cam[12];   /* row-major 3x4 [R | t]: x_cam = R x_world + t */
    float fx, fy, cx, cy;     /* pixels; pixel (i,j) has its centre at (i+1/2, j+1/2) */
    int32_t width, height;    /* 1..32768 */
    float near_z;             /* primitives with centre depth <= near_z are culled */
    int32_t reserved;
} linprim_camera;

/* Launch configuration. */
typedef struct linprim_tuning {
    int32_t tile;             /* screen tile edge in pixels: 8, 16 or 32 */
    int32_t sort_digit_bits;  /* radix-sort digit width, 4..8 (0 = 8); used with LINPRIM_FLAG_RADIX_SORT */
    int32_t flags;            /* LINPRIM_FLAG_* */
    int32_t reserved;
} linprim_tuning;

/* Count iterated / evaluated / intersected (pixel, primitive) pairs in
 * render_fwd (slower; for measurements). */
#define LINPRIM_FLAG_COUNTERS 1
/* linprim_preprocess does not write the camera table into view_ws: the
 * caller has done so with linprim_upload_views (e.g. before replaying a
 * captured graph whose camera poses change between replays; image sizes
 * must stay the same). */
#define LINPRIM_FLAG_VIEWS_RESIDENT 2
/* linprim_bin_sort orders the pairs with a global LSD radix sort of the
 * full (tile, depth) keys, sort_digit_bits per pass, instead of the default
 * per-tile sort (pairs counted and scattered per tile, each tile's list then
 * sorted by (depth, primitive)).  Both give the same order. */
#define LINPRIM_FLAG_RADIX_SORT 4
/* The variant without the ray-space approximation that the paper's appendix
 * on that approximation evaluates: each pixel ray leaves the camera centre
 * along ((i + 1/2 - cx)/fx, (j + 1/2 - cy)/fy, 1) and the chord is the
 * Euclidean length of its segment inside the camera-space primitive (true
 * ray / polytope intersection, no linearisation).  The pixel rectangle is
 * the box of the perspective-projected corners, and a primitive with any
 * corner at depth <= near_z is culled (its projection is undefined).  Depth
 * keys, sorting, compositing and Eq. 1 are unchanged.  The flag must be the
 * same in every call on one pair of workspaces. */
#define LINPRIM_FLAG_EXACT_RAYS 8
/* The 2D anti-aliasing filter of the paper's appendix on anti-aliasing
 * (filter size 0.1 pixel, App. G): in ray space, the corners that lie on
 * the primitive's tiling box move outward, parallel to the screen, by
 * 0.1 pixel (an octahedron's axis vector, which carries two mirrored
 * corners, by 0.05); every corner attaining an extreme moves, along both
 * axes if it attains two.  This enlarges the footprint and the chords of
 * small primitives; gradients pass through the constant shift.  Not
 * combinable with LINPRIM_FLAG_EXACT_RAYS (INVALID_ARG).  Same flag in
 * every call on one pair of workspaces. */
#define LINPRIM_FLAG_ANTIALIAS 16

/* Bytes of the per-view workspace (payloads, counts, offsets, tile ranges,
 * status) for n primitives of `type` over n_views cameras; 0 for invalid
 * arguments, including n * n_views >= 2^32. */
size_t linprim_view_workspace_size(int32_t type, int64_t n, const linprim_camera *cams,
                                   int32_t n_views, const linprim_tuning *tuning);

/* Bytes of the pair workspace (sort keys and values, double-buffered, sort
 * histograms and the per-pair gradient records of render_bwd) for up to
 * max_pairs (tile, primitive) pairs. */
size_t linprim_pair_workspace_size(int64_t max_pairs, const linprim_camera *cams, int32_t n_views,
                                   const linprim_tuning *tuning);

/* Sec. 3.2 "Preprocessing".  Writes, into view_ws, the render payload
 * (ray-space planes, or camera-space ones with LINPRIM_FLAG_EXACT_RAYS) of
 * every (view, primitive), its pixel and tile rectangles, depth
 * key and tile count, and the exclusive prefix sum of the tile counts (the
 * total is the pair count).  The binning quantities are computed in IEEE
 * double precision with a fixed evaluation order, so they are reproducible
 * bit for bit by any implementation that follows the same expressions.
 * cams: HOST array [n_views].  The same prims, cams, n_views and tuning
 * must be passed to every later call that uses this view_ws. */
int linprim_preprocess(const linprim_prims *prims, const linprim_camera *cams, int32_t n_views,
                       const linprim_tuning *tuning, void *view_ws, size_t view_ws_bytes, void *stream);

/* Writes the camera table of `cams` (HOST array) into view_ws, as
 * linprim_preprocess does unless LINPRIM_FLAG_VIEWS_RESIDENT is set.  The
 * camera values travel as kernel arguments, so the call is graph-capturable
 * and the host array may be reused as soon as it returns. */
int linprim_upload_views(const linprim_camera *cams, int32_t n_views, const linprim_tuning *tuning,
                         void *view_ws, size_t view_ws_bytes, int64_t n, int32_t type, void *stream);

/* Waits for `stream` and returns the pair count of the last preprocess. */
int linprim_pair_count(const void *view_ws, int64_t *n_pairs, void *stream);

/* Sec. 3.2 "Global Sorting and Tiling".  Orders the (tile, primitive)
 * pairs of every touched tile by key = (global tile << 32) | float32 bits of
 * the centre's camera depth, ties by primitive index, and writes every
 * tile's [start, end) range into view_ws.  By default the pairs are grouped
 * by tile with a stable LSD radix sort of the tile bits and each tile's
 * segment is sorted by (depth, primitive); with LINPRIM_FLAG_RADIX_SORT a
 * stable LSD radix sort of the full keys gives the same order.  If the pair count exceeds
 * max_pairs nothing is sorted, the overflow flag in view_ws is set and the
 * render calls leave their outputs untouched; linprim_read_status reports
 * it.  The sorted keys/values stay in pair_ws. */
int linprim_bin_sort(const linprim_prims *prims, const linprim_camera *cams, int32_t n_views,
                     const linprim_tuning *tuning, void *view_ws, size_t view_ws_bytes, void *pair_ws,
                     size_t pair_ws_bytes, int64_t max_pairs, void *stream);

/* Sec. 3.2 "Rasterization" and "Compositing".  For every pixel, walks its
 * tile's sorted list; a primitive whose pixel rectangle contains the pixel
 * contributes opacity o = min(1 - exp(-sigma * chord), 0.99), with the chord
 * the length of the pixel ray inside the ray-space primitive and sigma from
 * Eq. 1; C += T o rgb, T *= 1 - o, and the walk stops after T <= 1e-3.
 * Finally C += T bg.
 *   bg       HOST float[3] background colour
 *   out_rgb  [sum_v 3 H_v W_v] view-major, each view [3,H,W]
 *   out_T    [sum_v H_v W_v] final transmittance
 *   out_last [sum_v H_v W_v] one past the list position of the last blended
 *            primitive (the tile's list start if none) */
int linprim_render_fwd(const linprim_prims *prims, const linprim_camera *cams, int32_t n_views,
                       const linprim_tuning *tuning, const float *bg, const void *view_ws,
                       size_t view_ws_bytes, const void *pair_ws, size_t pair_ws_bytes, int64_t max_pairs,
                       float *out_rgb, float *out_T, int32_t *out_last, void *stream);

/* Sec. 3.4 and App. E.  Given grad_rgb = dL/dC (layout of out_rgb) and the
 * forward's out_T and out_last, walks every pixel's list backwards,
 * recomputing transmittance (no per-sample state is stored), and writes the
 * gradients with respect to the primitive features, summed over views.  The
 * density normaliser min(d) of Eq. 1 is held constant (App. G).  Gradients
 * are OVERWRITTEN; grad_sh has the layout of prims->sh.  Deterministic: no
 * floating-point atomics. */
int linprim_render_bwd(const linprim_prims *prims, const linprim_camera *cams, int32_t n_views,
                       const linprim_tuning *tuning, const float *bg, void *view_ws,
                       size_t view_ws_bytes, void *pair_ws, size_t pair_ws_bytes, int64_t max_pairs,
                       const float *out_T, const int32_t *out_last, const float *grad_rgb,
                       float *grad_means, float *grad_quats, float *grad_dists, float *grad_opacity,
                       float *grad_sh, void *stream);

/* The two stages of linprim_render_bwd, callable on their own (Sec. 3.4
 * "Rasterization Backpropagation" and "Preprocessing Backpropagation").
 * linprim_raster_bwd writes one gradient record per (tile, primitive) pair
 * into pair_ws: dL/d(plane coefficients of the payload), dL/d rgb and dL/d sigma
 * summed over the tile's pixels.  linprim_preprocess_bwd sums each
 * primitive's records in a fixed order (in place, in pair_ws) and carries
 * them to the features; outputs as in linprim_render_bwd.  It also leaves,
 * in view_ws, each visible (view, primitive)'s screen statistics that
 * linprim_accumulate_stats reads. */
int linprim_raster_bwd(const linprim_prims *prims, const linprim_camera *cams, int32_t n_views,
                       const linprim_tuning *tuning, const float *bg, const void *view_ws,
                       size_t view_ws_bytes, void *pair_ws, size_t pair_ws_bytes, int64_t max_pairs,
                       const float *out_T, const int32_t *out_last, const float *grad_rgb, void *stream);
int linprim_preprocess_bwd(const linprim_prims *prims, const linprim_camera *cams, int32_t n_views,
                           const linprim_tuning *tuning, void *view_ws, size_t view_ws_bytes,
                           void *pair_ws, size_t pair_ws_bytes, int64_t max_pairs, float *grad_means,
                           float *grad_quats, float *grad_dists, float *grad_opacity, float *grad_sh,
                           void *stream);

/* The optimisation step around the rasterizer (Sec. 3.4 "Optimization";
 * learning rates of App. G, Table "learning rates").
 *
 * linprim_l1_grad: for L = scale * sum_i |rgb_i - target_i| over `count`
 * floats, writes grad = dL/drgb = scale * sign(rgb - target) and, for each
 * block of 1024 elements, the block's share of L into
 * partial[ceil(count / 1024)] (summing the partials gives L; they are for
 * logging, the gradient does not need them).  All DEVICE pointers.
 * skip: NULL, or a DEVICE word read when the kernel runs; if it is non-zero
 * (linprim_step_guard's guard[0] after a pair overflow) nothing is written. */
int linprim_l1_grad(const float *rgb, const float *target, int64_t count, float scale, float *grad,
                    float *partial, const uint32_t *skip, void *stream);

/* One Adam step (Kingma & Ba; Sec. 3.4) over up to 8 parameter groups in
 * a single launch: m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2,
 * p -= lr (m / (1-b1^t)) / (sqrt(v / (1-b2^t)) + eps), then p is clamped to
 * [lo, hi] (use -inf/+inf for none; e.g. distances stay positive and
 * opacities inside [0, 1]).  groups: HOST array; the tensors are DEVICE
 * float32 arrays of `numel` elements; step t >= 1.
 *
 * period > 0 gives a group two learning rates: element i uses lr_tail when
 * (i mod period) >= head, else lr.  With the SH array [N][16][3] as one
 * group, period 48 and head 3 give the colour (degree-0) coefficients and
 * the higher-degree ones the separate rates of the learning-rate table in
 * App. G.  period 0 (head, lr_tail ignored): every element uses lr.
 * Errors: INVALID_ARG for n_groups outside [1, 8], numel < 0, a null array
 * with numel > 0, head outside [0, period]. */
typedef struct linprim_adam_group {
    float *param;
    const float *grad;
    float *exp_avg;
    float *exp_avg_sq;
    int64_t numel;
    float lr;
    float lo, hi;
    int32_t period;
    float lr_tail;
    int32_t head;
} linprim_adam_group;

int linprim_adam_step(const linprim_adam_group *groups, int32_t n_groups, float beta1, float beta2,
                      float eps, int32_t step, void *stream);

/* As linprim_adam_step, with the bias corrections 1 - beta1^t and
 * 1 - beta2^t read from DEVICE memory bias_corr[2] when the kernel runs, so
 * that one captured graph serves every step (the caller updates the two
 * floats between replays).  linprim_adam_step forms them as
 * (float)(1.0 - pow((double)beta, (double)t)); values formed the same way
 * give bit-identical updates.  skip: NULL, or a DEVICE word read when the
 * kernel runs; if it is non-zero no parameter or moment changes (a step
 * whose pair workspace overflowed has no valid gradient). */
int linprim_adam_step_dev(const linprim_adam_group *groups, int32_t n_groups, float beta1, float beta2,
                          float eps, const float *bias_corr, const uint32_t *skip, void *stream);

/* Guard of a captured training step (preprocess, bin_sort, render, loss,
 * backward, Adam replayed as one graph): enqueued after linprim_bin_sort, it
 * writes guard[0] = 1 if that bin_sort overflowed its pair capacity, else 0,
 * and ORs the same value into guard[1].  guard: DEVICE uint32[2], owned by
 * the caller, who zeroes guard[1] once and reads it after any number of
 * replays to learn whether one of them overflowed (the library never clears
 * it).  Passing guard as `skip` to the loss-gradient and Adam entry points
 * makes an overflowed step leave the parameters unchanged.  Arguments as
 * for linprim_render_fwd; errors INVALID_ARG, WORKSPACE_TOO_SMALL. */
int linprim_step_guard(const linprim_prims *prims, const linprim_camera *cams, int32_t n_views,
                       const linprim_tuning *tuning, const void *view_ws, size_t view_ws_bytes, uint32_t *guard,
                       void *stream);

/* Waits for `stream`; reports the pair count and whether the last bin_sort
 * overflowed its capacity (HOST outputs). */
int linprim_read_status(const void *view_ws, int64_t *pairs_needed, int32_t *overflow, void *stream);

/* Same as linprim_render_fwd, and adds the iterated / evaluated /
 * intersected (pixel, primitive) pair counts of this call to counters[0..2]
 * (DEVICE uint64[3], accumulated with atomics).  Iterated: list entries a
 * pixel walks up to its stop; evaluated: those whose pixel rectangle holds
 * the pixel; intersected: those with a positive chord. */
int linprim_render_fwd_counted(const linprim_prims *prims, const linprim_camera *cams, int32_t n_views,
                               const linprim_tuning *tuning, const float *bg, const void *view_ws,
                               size_t view_ws_bytes, const void *pair_ws, size_t pair_ws_bytes,
                               int64_t max_pairs, float *out_rgb, float *out_T, int32_t *out_last,
                               uint64_t *counters, void *stream);

/* linprim_render_fwd plus the depth map of the paper's appendix "Depth and
 * Surface Reconstruction": out_depth [sum_v H_v W_v] (DEVICE float,
 * layout of out_T) receives, per pixel, the distance along the pixel's
 * viewing ray to the first primitive at whose blending the cumulative
 * opacity 1 - T exceeds 0.5 (T drops below 0.5), measured to that
 * primitive's entry point: its entry depth in ray space (whose depth axis
 * is the distance from the camera), or with LINPRIM_FLAG_EXACT_RAYS the
 * entry point's distance along the true pixel ray; 0 where 1 - T never
 * exceeds 0.5.  The accumulated-opacity (alpha) channel is 1 - out_T. */
int linprim_render_fwd_depth(const linprim_prims *prims, const linprim_camera *cams, int32_t n_views,
                             const linprim_tuning *tuning, const float *bg, const void *view_ws,
                             size_t view_ws_bytes, const void *pair_ws, size_t pair_ws_bytes,
                             int64_t max_pairs, float *out_rgb, float *out_T, int32_t *out_last,
                             float *out_depth, void *stream);

/* ------------------------------------------------------------------------
 * Adaptive population control (Sec. 3.4 "Adaptive Population Control";
 * thresholds in App. G).
 * ------------------------------------------------------------------------ */

/* Adds, for every primitive, the statistics of the last backward pass on
 * these workspaces (linprim_render_bwd or linprim_preprocess_bwd, ray-space
 * model): over the views in which it touches a tile, the norm of its
 * view-space positional gradient (dL/d ray-space centre x, y with the
 * primitive's ray-space offsets held fixed, per unit of normalised device
 * coordinates: x scaled by W/2, y by H/2) into grad_accum, the number of
 * such views into count, and the largest screen radius (half the larger
 * side of the projected bounding box, pixels) into max_radius.  All three
 * DEVICE arrays [n] are read-modify-written (zero them to start).  With
 * LINPRIM_FLAG_EXACT_RAYS the gradient norms are 0 (the quantity belongs to
 * the ray-space model); counts and radii are still kept. */
int linprim_accumulate_stats(const linprim_prims *prims, const linprim_camera *cams, int32_t n_views,
                             const linprim_tuning *tuning, const void *view_ws, size_t view_ws_bytes,
                             float *grad_accum, int32_t *count, float *max_radius, void *stream);

/* Thresholds of the densify / prune pass (App. G's values in brackets).
 * Every decision is taken in float32. */
typedef struct linprim_densify_params {
    float grad_threshold;      /* mean positional gradient above which a primitive densifies [1.5e-4] */
    float min_opacity;         /* primitives with a smaller opacity are removed [0.025] */
    float max_size_frac;       /* primitives larger than this fraction of the extent are removed [0.4] */
    float max_screen_radius;   /* originals whose largest screen radius exceeds this are removed [20 px] */
    float clone_size_frac;     /* candidates smaller than this fraction of the extent are cloned [0.01] */
    float split_shrink;        /* split children's distances are divided by this [1.2] */
    float extent;              /* scene extent, world units */
    int32_t reserved;
} linprim_densify_params;

/* The primitives and, optionally, their Adam moments: DEVICE arrays with
 * the layouts of linprim_prims (means [n,3], quats [n,4], dists [n,3|4],
 * opacity [n], sh [n,(deg+1)^2,3]); exp_avg / exp_avg_sq in the same order
 * and shapes, all NULL for none. */
typedef struct linprim_state {
    float *means, *quats, *dists, *opacity, *sh;
    float *exp_avg[5];
    float *exp_avg_sq[5];
} linprim_state;

/* Bytes of the densify workspace for n primitives. */
size_t linprim_densify_workspace_size(int64_t n);

/* Decides, per primitive, from its size (octahedron: longest axis 2 max d;
 * tetrahedron: sqrt(2) times the distance to the furthest corner), its mean
 * positional gradient grad_accum / count, its opacity and max_radius:
 *   candidate: mean gradient > grad_threshold;
 *   a candidate with size < clone_size_frac * extent is cloned (same
 *   features, zero moments), a larger one is replaced by two children
 *   (distances / split_shrink, zero moments, positions drawn as below);
 *   removed: opacity < min_opacity, size > max_size_frac * extent (a split
 *   child with its reduced size), or, for originals, max_radius >
 *   max_screen_radius.
 * Writes the plan into ws and returns, in *n_out (HOST), the number of
 * primitives after the pass.  Waits for `stream`. */
int linprim_densify_plan(int32_t type, int64_t n, const float *dists, const float *opacity,
                         const float *grad_accum, const int32_t *count, const float *max_radius,
                         const linprim_densify_params *params, void *ws, size_t ws_bytes, int64_t *n_out,
                         void *stream);

/* Writes the n_out primitives of the plan into dst (DEVICE arrays sized
 * for n_out rows, not overlapping src): for each input primitive in order,
 * the original (with its moments) or its two split children, then its
 * clone.  Split child c of primitive i is placed at mu + R (d * z) for an
 * octahedron (standard deviations equal to its distances along its own
 * axes, then rotated) or at mu + (max d / 2) z for a tetrahedron, with z =
 * normals[i][c][0..2] (DEVICE float [n][2][3], standard normal draws the
 * caller provides).  dst moments are written when dst.exp_avg[0] is not
 * NULL (zero for new primitives, copied otherwise). */
int linprim_densify_apply(int32_t type, int32_t sh_degree, int64_t n, const linprim_state *src,
                          const float *normals, const float *grad_accum, const int32_t *count,
                          const float *max_radius, const linprim_densify_params *params, const void *ws,
                          size_t ws_bytes, const linprim_state *dst, int64_t n_out, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid hipMalloc): linprim_densify_plan
 * and linprim_densify_apply in one call, with the plan's block sums in a
 * scratch array the library holds in device memory (8 bytes per 1,024
 * primitives of up to LINPRIM_NOALLOC_MAX_PRIMS, about 64 KiB per device,
 * kept until the process ends) instead of a caller workspace.  It calls no
 * allocating routine.  dst: DEVICE arrays of dst_rows rows (3 n rows always
 * suffice); *n_out (HOST) receives the number of primitives after the pass;
 * if it exceeds dst_rows, dst is left untouched and WORKSPACE_TOO_SMALL is
 * returned.  Waits for `stream` once, between plan and apply.  Errors:
 * WORKSPACE_TOO_SMALL for n > LINPRIM_NOALLOC_MAX_PRIMS (checked first) or
 * dst_rows < *n_out; INVALID_ARG as for the two calls it combines.  Every
 * call on one device shares that device's scratch: calls that overlap on
 * one device (other streams, other host threads) race. */
#define LINPRIM_NOALLOC_MAX_PRIMS 8388608
int linprim_densify_noalloc(int32_t type, int32_t sh_degree, int64_t n, const linprim_state *src,
                            const float *normals, const float *grad_accum, const int32_t *count,
                            const float *max_radius, const linprim_densify_params *params,
                            const linprim_state *dst, int64_t dst_rows, int64_t *n_out, void *stream);

/* ------------------------------------------------------------------------
 * LinPrim-MCMC (Sec. 3.4 "LinPrim-MCMC"): GS-MCMC's relocation and noise
 * steps for octahedra treated as Gaussians with standard deviations d / 2.6.
 * Octahedra only (other types: INVALID_ARG).
 * ------------------------------------------------------------------------ */

/* Bytes of the relocation workspace for n primitives. */
size_t linprim_mcmc_workspace_size(int64_t n);

/* In place on `state` (DEVICE, moments optional): every dead primitive
 * (opacity <= 0.005) becomes a copy of a live source drawn with probability
 * proportional to its opacity -- integer weights floor(alpha 2^32), the k-th
 * dead primitive (index order) taking the first index whose inclusive
 * weight prefix exceeds floor(total * rand[k] / 2^32), rand DEVICE uint32[n]
 * from the caller.  A source drawn c times first becomes one of
 * N = min(c + 1, 51) copies: opacity 1 - (1 - alpha)^(1/N) (clamped to
 * [0.005, 1 - 2^-23]) and distances times
 * alpha / sum_{i=1}^{N} sum_{k=0}^{i-1} C(i-1,k) (-1)^k alpha_new^(k+1) / sqrt(k+1).
 * Moments of sources and relocated primitives are reset to zero.  Nothing
 * happens if no primitive is alive. */
int linprim_mcmc_relocate(int32_t type, int32_t sh_degree, int64_t n, const linprim_state *state,
                          const uint32_t *rand, void *ws, size_t ws_bytes, void *stream);

/* GS-MCMC's growth step: draws n_add sources (n_add <= n) among the first
 * n rows of `state` exactly as linprim_mcmc_relocate draws them (rand
 * DEVICE uint32[n_add]), applies the same source update, and writes the
 * copies to rows n .. n + n_add - 1 (the arrays must hold n + n_add rows;
 * the caller copies the first n).  The caller picks n_add (GS-MCMC: grow by
 * 5% per step up to a cap).  ws: linprim_mcmc_workspace_size(n). */
int linprim_mcmc_add(int32_t type, int32_t sh_degree, int64_t n, int64_t n_add, const linprim_state *state,
                     const uint32_t *rand, void *ws, size_t ws_bytes, void *stream);

/* Waits for `stream` and returns the number of dead primitives the last
 * linprim_mcmc_relocate on ws found (all of them were relocated if any
 * primitive was alive). */
int linprim_mcmc_dead_count(const void *ws, size_t ws_bytes, int64_t n, int64_t *n_dead, void *stream);

/* means += noise_lr * lr_means * s(1 - alpha) * R S^2 R^T eps, S = diag(d / 2.6),
 * s(x) = 1 / (1 + exp(-100 (x - 0.995))), eps = normals (DEVICE float [n][3],
 * standard normal draws from the caller). */
int linprim_mcmc_noise(int32_t type, int64_t n, const linprim_state *state, const float *normals, float lr_means,
                       float noise_lr, void *stream);

/* ------------------------------------------------------------------------
 * Photometric loss of the optimisation (Sec. 3.4 "Optimization": the loss
 * of 3DGS, an L1 and an SSIM term).  Per view, with n = 3 H W,
 *   L_v = (1 - lambda) sum |C - T| / n + lambda (1 - sum s / n),
 *   s = (2 mx my + C1)(2 sxy + C2) / ((mx^2 + my^2 + C1)(sxx + syy + C2)),
 * local statistics mx, my, sxx, syy, sxy of each channel by an 11 x 11
 * Gaussian window (standard deviation 1.5, normalised), zero padding at the
 * border, C1 = 0.01^2, C2 = 0.03^2; the loss of a batch is sum_v L_v
 * (3DGS's weight: lambda = 0.2).
 * ------------------------------------------------------------------------ */

/* Bytes of the loss workspace (per-block partial sums and three per-pixel
 * derivative maps of the largest view). */
size_t linprim_loss_workspace_size(const linprim_camera *cams, int32_t n_views);

/* dL/dC for the packed view-major images rgb and target (DEVICE, layout of
 * linprim_render_fwd's out_rgb) into grad (DEVICE, same layout; may not
 * alias the inputs); the partial sums of the loss stay in ws.  sign(0) = 0
 * in the L1 term.  Graph-capturable.  skip: as for linprim_l1_grad. */
int linprim_loss_grad(const float *rgb, const float *target, const linprim_camera *cams, int32_t n_views,
                      float lambda, void *ws, size_t ws_bytes, float *grad, const uint32_t *skip, void *stream);

/* Waits for `stream` and returns, in *loss (HOST), sum_v L_v of the last
 * linprim_loss_grad on ws, the partial sums added in double precision. */
int linprim_loss_value(const void *ws, size_t ws_bytes, const linprim_camera *cams, int32_t n_views, float lambda,
                       double *loss, void *stream);

/* Static description of an error code. */
const char *linprim_strerror(int code);

/* Device pointers into the workspaces, for tests and diagnostics:
 * payload [n_views*n][32] (float; words 0..3 are the int pixel rectangle
 * i0, j0, i1, j1; a culled slot, tiles_touched = 0, has no valid record),
 * depth_keys [n_views*n] u32, tiles_touched [n_views*n] u32, offsets
 * [n_views*n] u32, sorted keys
 * [max_pairs] u64 and values [max_pairs] u32 (first n_pairs valid),
 * ranges [total tiles] (u32 start, u32 end), and the two render orders
 * [total tiles] u32 written by linprim_bin_sort (the tile taken by each wave
 * position: forward, lists of more than 128 pairs first, then those of more
 * than 72, then the others, each part in tile order; backward, by classes of
 * list length, longest first, each class in tile order; the exact variant's
 * forward takes the backward order).  Any out-pointer may be NULL. */
int linprim_debug_pointers(const linprim_prims *prims, const linprim_camera *cams, int32_t n_views,
                           const linprim_tuning *tuning, const void *view_ws, const void *pair_ws,
                           int64_t max_pairs, void **payload, void **depth_keys, void **tiles_touched,
                           void **offsets, void **keys, void **values, void **ranges, void **order_fwd,
                           void **order_bwd);

#ifdef __cplusplus
}
#endif

#endif /* LINPRIM_H */
