// abi.hip -- the extern "C" entry points of liblinprim.so: argument
// validation, workspace layouts and launch order.  Every call enqueues on
// the caller's stream; only linprim_pair_count / linprim_read_status wait.
#include <stdlib.h>
#include <string.h>

#include "linprim_common.h"

namespace linprim {

int key_tile_bits(int64_t n_tiles_total) {
    int b = 1;
    while ((int64_t(1) << b) < n_tiles_total) ++b;
    return b;
}

static int64_t total_tiles(const linprim_camera* cams, int32_t n_views, int tile) {
    int64_t t = 0;
    for (int v = 0; v < n_views; ++v)
        t += (int64_t)((cams[v].width + tile - 1) / tile) * ((cams[v].height + tile - 1) / tile);
    return t;
}

ViewLayout view_layout(int64_t n, const linprim_camera* cams, int32_t n_views, int tile) {
    ViewLayout L;
    L.n = n;
    L.n_views = n_views;
    L.n_tiles_total = total_tiles(cams, n_views, tile);
    const int64_t vn = n * n_views;
    L.scan_blocks = (vn + kScanItems - 1) / kScanItems;
    size_t off = 0;
    L.status = off; off = align256(off + sizeof(Status));
    L.views = off; off = align256(off + sizeof(ViewInfo) * (size_t)n_views);
    L.payload = off; off = align256(off + (size_t)vn * kRecordWords * 4);
    L.depth_keys = off; off = align256(off + (size_t)vn * 4);
    L.tiles = off; off = align256(off + (size_t)vn * 4);
    L.offsets = off; off = align256(off + (size_t)vn * 4);
    L.block_sums = off; off = align256(off + (size_t)(L.scan_blocks + 1) * 16);   // tile sums, visible counts
    L.ranges = off; off = align256(off + (size_t)L.n_tiles_total * 8);
    L.big = off; off = align256(off + (size_t)vn * 4);
    L.long_list = off; off = align256(off + (size_t)L.n_tiles_total * 4);
    L.vis = off; off = align256(off + (size_t)vn * 4);
    L.stats = off; off = align256(off + (size_t)vn * 8);
    L.order = off; off = align256(off + (size_t)L.n_tiles_total * 4);
    L.order_bwd = off; off = align256(off + (size_t)L.n_tiles_total * 4);
    L.order_sums = off;
    const int64_t oi = order_items(L.n_tiles_total);
    off = align256(off + (size_t)(((L.n_tiles_total + oi - 1) / oi) * kOrderClasses + 1) * 4);
    L.huge = off; off = align256(off + (size_t)vn * 4);
    L.trect = off; off = align256(off + (size_t)vn * 8);
    L.total = off;
    return L;
}

PairLayout pair_layout(int64_t max_pairs, int digit_bits, int tile) {
    (void)digit_bits;
    const int nq = (tile / 8) * (tile / 8);
    PairLayout P;
    P.capacity = max_pairs;
    P.sort_blocks = (max_pairs + kSortTile - 1) / kSortTile;
    size_t off = 0;
    P.keys_a = off; off = align256(off + (size_t)max_pairs * 8);
    P.keys_b = off; off = align256(off + (size_t)max_pairs * 8);
    P.vals_a = off; off = align256(off + (size_t)max_pairs * 4);
    P.vals_b = off; off = align256(off + (size_t)max_pairs * 4);
    P.hist = off; off = align256(off + ((size_t)256 * P.sort_blocks + 256) * 4);
    P.grads = off; off = align256(off + (size_t)max_pairs * nq * kGradWords * 4);
    P.total = off;
    return P;
}

hipError_t launch_render_fwd_ex(const ViewLayout& L, const char* vws, const PairLayout& P, const char* pws,
                                int result_in_b, int type, bool exact, int tile, int32_t n_views, const float bg[3],
                                float* out_rgb, float* out_T, int32_t* out_last, float* out_depth,
                                const float* means, unsigned long long* counters, hipStream_t stream);

}  // namespace linprim

using namespace linprim;

namespace {

bool valid_tile(int t) { return t == 8 || t == 16 || t == 32; }

int tile_of(const linprim_tuning* tu) { return tu ? tu->tile : 16; }

int digit_of(const linprim_tuning* tu) {
    const int d = tu ? tu->sort_digit_bits : 0;
    return d == 0 ? 8 : d;
}

bool valid_tuning(const linprim_tuning* tu) {
    if (!valid_tile(tile_of(tu))) return false;
    // the anti-aliasing filter belongs to the ray-space model
    if (tu && (tu->flags & LINPRIM_FLAG_EXACT_RAYS) && (tu->flags & LINPRIM_FLAG_ANTIALIAS)) return false;
    const int d = digit_of(tu);
    return d >= 4 && d <= 8;
}

bool valid_cams(const linprim_camera* cams, int32_t n_views) {
    if (!cams || n_views < 1 || n_views > kMaxViews) return false;
    for (int v = 0; v < n_views; ++v)
        if (cams[v].width < 1 || cams[v].height < 1 || cams[v].width > 32768 || cams[v].height > 32768) return false;
    return true;
}

// (view, primitive) slots are indexed with 32-bit integers in the lists the
// scan builds.
bool valid_slots(int64_t n, int32_t n_views) { return n * (int64_t)n_views < (int64_t(1) << 32); }

bool valid_prims(const linprim_prims* p) {
    if (!p) return false;
    if (p->type != LINPRIM_OCTAHEDRON && p->type != LINPRIM_TETRAHEDRON) return false;
    if (p->sh_degree < 0 || p->sh_degree > 3) return false;
    if (p->n < 0 || p->n >= (int64_t(1) << 31)) return false;
    if (p->n > 0 && (!p->means || !p->quats || !p->dists || !p->opacity || !p->sh)) return false;
    return true;
}

// Architecture check, answered once per device (the answer is cached so
// that calls made under stream capture issue no device queries).
int check_device() {
    static int verdict[64];   // 0 unknown, 1 gfx950, 2 other
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return LINPRIM_ERR_HIP;
    if (dev < 0 || dev >= 64) return LINPRIM_ERR_DEVICE;
    if (verdict[dev] == 0) {
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return LINPRIM_ERR_HIP;
        verdict[dev] = (strncmp(prop.gcnArchName, "gfx950", 6) == 0) ? 1 : 2;
    }
    return verdict[dev] == 1 ? LINPRIM_OK : LINPRIM_ERR_DEVICE;
}

int hip_status(hipError_t e) { return e == hipSuccess ? LINPRIM_OK : LINPRIM_ERR_HIP; }

// The bin_sort call decides in which buffer the sorted pairs end (the
// parity of the number of digit passes); the render calls recompute it.
bool radix_sort(const linprim_tuning* tu) { return tu && (tu->flags & LINPRIM_FLAG_RADIX_SORT); }

bool exact_rays(const linprim_tuning* tu) { return tu && (tu->flags & LINPRIM_FLAG_EXACT_RAYS); }

bool antialias(const linprim_tuning* tu) { return tu && (tu->flags & LINPRIM_FLAG_ANTIALIAS); }

int result_buffer(const ViewLayout& L, const linprim_tuning* tu) {
    return sorted_buffer(L.n_tiles_total, radix_sort(tu), digit_of(tu));
}

}  // namespace

extern "C" {

size_t linprim_view_workspace_size(int32_t type, int64_t n, const linprim_camera* cams, int32_t n_views,
                                   const linprim_tuning* tuning) {
    if ((type != LINPRIM_OCTAHEDRON && type != LINPRIM_TETRAHEDRON) || n < 0 || !valid_cams(cams, n_views) ||
        !valid_tuning(tuning) || !valid_slots(n, n_views))
        return 0;
    return view_layout(n, cams, n_views, tile_of(tuning)).total;
}

size_t linprim_pair_workspace_size(int64_t max_pairs, const linprim_camera* cams, int32_t n_views,
                                   const linprim_tuning* tuning) {
    if (max_pairs < 0 || max_pairs >= (int64_t(1) << 31) || !valid_cams(cams, n_views) || !valid_tuning(tuning))
        return 0;
    return pair_layout(max_pairs, digit_of(tuning), tile_of(tuning)).total;
}

int linprim_preprocess(const linprim_prims* prims, const linprim_camera* cams, int32_t n_views,
                       const linprim_tuning* tuning, void* view_ws, size_t view_ws_bytes, void* stream) {
    if (!valid_prims(prims) || !valid_cams(cams, n_views) || !valid_tuning(tuning) || !view_ws ||
        !valid_slots(prims->n, n_views))
        return LINPRIM_ERR_INVALID_ARG;
    const int tile = tile_of(tuning);
    const ViewLayout L = view_layout(prims->n, cams, n_views, tile);
    if (view_ws_bytes < L.total) return LINPRIM_ERR_WORKSPACE;
    if (int rc = check_device()) return rc;
    hipStream_t s = (hipStream_t)stream;
    char* ws = (char*)view_ws;
    const bool resident = tuning && (tuning->flags & LINPRIM_FLAG_VIEWS_RESIDENT);
    hipError_t e = launch_preprocess(*prims, n_views, tile, exact_rays(tuning), antialias(tuning), L, ws, s,
                                     resident ? nullptr : cams);
    if (e == hipSuccess) e = launch_scan(L, ws, tile, s);
    return hip_status(e);
}

int linprim_upload_views(const linprim_camera* cams, int32_t n_views, const linprim_tuning* tuning, void* view_ws,
                         size_t view_ws_bytes, int64_t n, int32_t type, void* stream) {
    if (!valid_cams(cams, n_views) || !valid_tuning(tuning) || !view_ws || n < 0 || !valid_slots(n, n_views) ||
        (type != LINPRIM_OCTAHEDRON && type != LINPRIM_TETRAHEDRON))
        return LINPRIM_ERR_INVALID_ARG;
    const int tile = tile_of(tuning);
    const ViewLayout L = view_layout(n, cams, n_views, tile);
    if (view_ws_bytes < L.total) return LINPRIM_ERR_WORKSPACE;
    return hip_status(launch_store_views(cams, n_views, tile,
                                         reinterpret_cast<ViewInfo*>((char*)view_ws + L.views), (hipStream_t)stream));
}

int linprim_pair_count(const void* view_ws, int64_t* n_pairs, void* stream) {
    if (!view_ws || !n_pairs) return LINPRIM_ERR_INVALID_ARG;
    Status st;
    hipStream_t s = (hipStream_t)stream;
    if (hipMemcpyAsync(&st, view_ws, sizeof(Status), hipMemcpyDeviceToHost, s) != hipSuccess) return LINPRIM_ERR_HIP;
    if (hipStreamSynchronize(s) != hipSuccess) return LINPRIM_ERR_HIP;
    *n_pairs = (int64_t)st.n_pairs;
    return LINPRIM_OK;
}

// Common validation of the calls that follow preprocess: rebuilds both
// layouts and checks the workspace sizes.
static int prepare(const linprim_prims* prims, const linprim_camera* cams, int32_t n_views,
                   const linprim_tuning* tuning, size_t view_ws_bytes, size_t pair_ws_bytes, int64_t max_pairs,
                   ViewLayout& L, PairLayout& P) {
    if (!valid_prims(prims) || !valid_cams(cams, n_views) || !valid_tuning(tuning) || max_pairs < 0 ||
        max_pairs >= (int64_t(1) << 31) || !valid_slots(prims->n, n_views))
        return LINPRIM_ERR_INVALID_ARG;
    L = view_layout(prims->n, cams, n_views, tile_of(tuning));
    P = pair_layout(max_pairs, digit_of(tuning), tile_of(tuning));
    if (view_ws_bytes < L.total || pair_ws_bytes < P.total) return LINPRIM_ERR_WORKSPACE;
    return LINPRIM_OK;
}

int linprim_bin_sort(const linprim_prims* prims, const linprim_camera* cams, int32_t n_views,
                     const linprim_tuning* tuning, void* view_ws, size_t view_ws_bytes, void* pair_ws,
                     size_t pair_ws_bytes, int64_t max_pairs, void* stream) {
    if (!view_ws || !pair_ws) return LINPRIM_ERR_INVALID_ARG;
    ViewLayout L;
    PairLayout P;
    if (int rc = prepare(prims, cams, n_views, tuning, view_ws_bytes, pair_ws_bytes, max_pairs, L, P)) return rc;
    int in_b = 0;
    hipError_t e = launch_bin_sort(L, (char*)view_ws, P, (char*)pair_ws, radix_sort(tuning), tile_of(tuning),
                                   digit_of(tuning), n_views,
                                   cams, (hipStream_t)stream, &in_b);
    return hip_status(e);
}

static int render_fwd_common(const linprim_prims* prims, const linprim_camera* cams, int32_t n_views,
                             const linprim_tuning* tuning, const float* bg, const void* view_ws, size_t view_ws_bytes,
                             const void* pair_ws, size_t pair_ws_bytes, int64_t max_pairs, float* out_rgb,
                             float* out_T, int32_t* out_last, float* out_depth, uint64_t* counters, void* stream) {
    if (!bg || !view_ws || !pair_ws || !out_rgb || !out_T || !out_last) return LINPRIM_ERR_INVALID_ARG;
    ViewLayout L;
    PairLayout P;
    if (int rc = prepare(prims, cams, n_views, tuning, view_ws_bytes, pair_ws_bytes, max_pairs, L, P)) return rc;
    const int in_b = result_buffer(L, tuning);
    hipError_t e = launch_render_fwd_ex(L, (const char*)view_ws, P, (const char*)pair_ws, in_b, prims->type,
                                        exact_rays(tuning), tile_of(tuning), n_views, bg, out_rgb, out_T, out_last,
                                        out_depth, prims->means, reinterpret_cast<unsigned long long*>(counters),
                                        (hipStream_t)stream);
    return hip_status(e);
}

int linprim_render_fwd(const linprim_prims* prims, const linprim_camera* cams, int32_t n_views,
                       const linprim_tuning* tuning, const float* bg, const void* view_ws, size_t view_ws_bytes,
                       const void* pair_ws, size_t pair_ws_bytes, int64_t max_pairs, float* out_rgb, float* out_T,
                       int32_t* out_last, void* stream) {
    return render_fwd_common(prims, cams, n_views, tuning, bg, view_ws, view_ws_bytes, pair_ws, pair_ws_bytes,
                             max_pairs, out_rgb, out_T, out_last, nullptr, nullptr, stream);
}

int linprim_render_fwd_depth(const linprim_prims* prims, const linprim_camera* cams, int32_t n_views,
                             const linprim_tuning* tuning, const float* bg, const void* view_ws, size_t view_ws_bytes,
                             const void* pair_ws, size_t pair_ws_bytes, int64_t max_pairs, float* out_rgb,
                             float* out_T, int32_t* out_last, float* out_depth, void* stream) {
    if (!out_depth) return LINPRIM_ERR_INVALID_ARG;
    return render_fwd_common(prims, cams, n_views, tuning, bg, view_ws, view_ws_bytes, pair_ws, pair_ws_bytes,
                             max_pairs, out_rgb, out_T, out_last, out_depth, nullptr, stream);
}

int linprim_render_fwd_counted(const linprim_prims* prims, const linprim_camera* cams, int32_t n_views,
                               const linprim_tuning* tuning, const float* bg, const void* view_ws,
                               size_t view_ws_bytes, const void* pair_ws, size_t pair_ws_bytes, int64_t max_pairs,
                               float* out_rgb, float* out_T, int32_t* out_last, uint64_t* counters, void* stream) {
    if (!counters) return LINPRIM_ERR_INVALID_ARG;
    return render_fwd_common(prims, cams, n_views, tuning, bg, view_ws, view_ws_bytes, pair_ws, pair_ws_bytes,
                             max_pairs, out_rgb, out_T, out_last, nullptr, counters, stream);
}

int linprim_render_bwd(const linprim_prims* prims, const linprim_camera* cams, int32_t n_views,
                       const linprim_tuning* tuning, const float* bg, void* view_ws, size_t view_ws_bytes,
                       void* pair_ws, size_t pair_ws_bytes, int64_t max_pairs, const float* out_T,
                       const int32_t* out_last, const float* grad_rgb, float* grad_means, float* grad_quats,
                       float* grad_dists, float* grad_opacity, float* grad_sh, void* stream) {
    if (!bg || !view_ws || !pair_ws || !out_T || !out_last || !grad_rgb) return LINPRIM_ERR_INVALID_ARG;
    if (prims && prims->n > 0 && (!grad_means || !grad_quats || !grad_dists || !grad_opacity || !grad_sh))
        return LINPRIM_ERR_INVALID_ARG;
    ViewLayout L;
    PairLayout P;
    if (int rc = prepare(prims, cams, n_views, tuning, view_ws_bytes, pair_ws_bytes, max_pairs, L, P)) return rc;
    const int in_b = result_buffer(L, tuning);
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = launch_render_bwd(L, (const char*)view_ws, P, (char*)pair_ws, in_b, prims->type,
                                     exact_rays(tuning), tile_of(tuning), n_views, bg, out_T, out_last, grad_rgb, s);
    if (e == hipSuccess)
        e = launch_preprocess_bwd(*prims, n_views, tile_of(tuning), exact_rays(tuning), antialias(tuning), L, (const char*)view_ws, P,
                                  (const char*)pair_ws,
                                  grad_means, grad_quats, grad_dists, grad_opacity, grad_sh, s);
    return hip_status(e);
}

int linprim_raster_bwd(const linprim_prims* prims, const linprim_camera* cams, int32_t n_views,
                       const linprim_tuning* tuning, const float* bg, const void* view_ws, size_t view_ws_bytes,
                       void* pair_ws, size_t pair_ws_bytes, int64_t max_pairs, const float* out_T,
                       const int32_t* out_last, const float* grad_rgb, void* stream) {
    if (!bg || !view_ws || !pair_ws || !out_T || !out_last || !grad_rgb) return LINPRIM_ERR_INVALID_ARG;
    ViewLayout L;
    PairLayout P;
    if (int rc = prepare(prims, cams, n_views, tuning, view_ws_bytes, pair_ws_bytes, max_pairs, L, P)) return rc;
    const int in_b = result_buffer(L, tuning);
    return hip_status(launch_render_bwd(L, (const char*)view_ws, P, (char*)pair_ws, in_b, prims->type,
                                        exact_rays(tuning), tile_of(tuning), n_views, bg, out_T, out_last, grad_rgb,
                                        (hipStream_t)stream));
}

int linprim_preprocess_bwd(const linprim_prims* prims, const linprim_camera* cams, int32_t n_views,
                           const linprim_tuning* tuning, void* view_ws, size_t view_ws_bytes,
                           void* pair_ws, size_t pair_ws_bytes, int64_t max_pairs, float* grad_means,
                           float* grad_quats, float* grad_dists, float* grad_opacity, float* grad_sh, void* stream) {
    if (!view_ws || !pair_ws) return LINPRIM_ERR_INVALID_ARG;
    if (prims && prims->n > 0 && (!grad_means || !grad_quats || !grad_dists || !grad_opacity || !grad_sh))
        return LINPRIM_ERR_INVALID_ARG;
    ViewLayout L;
    PairLayout P;
    if (int rc = prepare(prims, cams, n_views, tuning, view_ws_bytes, pair_ws_bytes, max_pairs, L, P)) return rc;
    return hip_status(launch_preprocess_bwd(*prims, n_views, tile_of(tuning), exact_rays(tuning), antialias(tuning), L,
                                            (const char*)view_ws, P,
                                            (const char*)pair_ws, grad_means, grad_quats, grad_dists, grad_opacity,
                                            grad_sh, (hipStream_t)stream));
}

int linprim_accumulate_stats(const linprim_prims* prims, const linprim_camera* cams, int32_t n_views,
                             const linprim_tuning* tuning, const void* view_ws, size_t view_ws_bytes,
                             float* grad_accum, int32_t* count, float* max_radius, void* stream) {
    if (!valid_prims(prims) || !valid_cams(cams, n_views) || !valid_tuning(tuning) || !view_ws ||
        !valid_slots(prims->n, n_views))
        return LINPRIM_ERR_INVALID_ARG;
    if (prims->n > 0 && (!grad_accum || !count || !max_radius)) return LINPRIM_ERR_INVALID_ARG;
    const ViewLayout L = view_layout(prims->n, cams, n_views, tile_of(tuning));
    if (view_ws_bytes < L.total) return LINPRIM_ERR_WORKSPACE;
    return hip_status(launch_accumulate_stats(prims->n, n_views, L, (const char*)view_ws, grad_accum, count,
                                              max_radius, (hipStream_t)stream));
}

size_t linprim_densify_workspace_size(int64_t n) {
    if (n < 0 || n >= (int64_t(1) << 31)) return 0;
    const int64_t nb = (n + kDensifyItems - 1) / kDensifyItems;
    return align256((size_t)(nb + 1) * 8);
}

static bool finite_f(float x) { return x - x == 0.0f; }   // false for inf and NaN

static bool valid_densify(const linprim_densify_params* dp) {
    return dp && dp->split_shrink > 0.0f && dp->extent > 0.0f && finite_f(dp->extent) &&
           finite_f(dp->split_shrink) && finite_f(dp->grad_threshold) && finite_f(dp->min_opacity) &&
           finite_f(dp->max_size_frac) && finite_f(dp->max_screen_radius) && finite_f(dp->clone_size_frac);
}

static DensifyParams densify_params(const linprim_densify_params* dp) {
    return {dp->grad_threshold, dp->min_opacity, dp->max_size_frac, dp->max_screen_radius, dp->clone_size_frac,
            dp->split_shrink};
}

int linprim_densify_plan(int32_t type, int64_t n, const float* dists, const float* opacity, const float* grad_accum,
                         const int32_t* count, const float* max_radius, const linprim_densify_params* params,
                         void* ws, size_t ws_bytes, int64_t* n_out, void* stream) {
    if ((type != LINPRIM_OCTAHEDRON && type != LINPRIM_TETRAHEDRON) || n < 0 || n >= (int64_t(1) << 31) || !ws ||
        !n_out || !valid_densify(params))
        return LINPRIM_ERR_INVALID_ARG;
    if (n > 0 && (!dists || !opacity || !grad_accum || !count || !max_radius)) return LINPRIM_ERR_INVALID_ARG;
    if (ws_bytes < linprim_densify_workspace_size(n)) return LINPRIM_ERR_WORKSPACE;
    if (int rc = check_device()) return rc;
    hipStream_t s = (hipStream_t)stream;
    int64_t* bs = (int64_t*)ws;
    hipError_t e = launch_densify_plan(type, n, dists, opacity, grad_accum, count, max_radius,
                                       densify_params(params), params->extent, bs, s);
    if (e != hipSuccess) return LINPRIM_ERR_HIP;
    const int64_t nb = (n + kDensifyItems - 1) / kDensifyItems;
    int64_t total = 0;
    if (hipMemcpyAsync(&total, bs + nb, sizeof(int64_t), hipMemcpyDeviceToHost, s) != hipSuccess) return LINPRIM_ERR_HIP;
    if (hipStreamSynchronize(s) != hipSuccess) return LINPRIM_ERR_HIP;
    *n_out = total;
    return LINPRIM_OK;
}

static bool state_ok(const linprim_state* st, int64_t rows) {
    if (!st) return false;
    if (rows == 0) return true;
    if (!st->means || !st->quats || !st->dists || !st->opacity || !st->sh) return false;
    const bool any = st->exp_avg[0] != nullptr;
    for (int f = 0; f < 5; ++f)
        if ((st->exp_avg[f] != nullptr) != any || (st->exp_avg_sq[f] != nullptr) != any) return false;
    return true;
}

static StateSet state_set(const linprim_state* st) {
    StateSet S;
    float* p[5] = {st->means, st->quats, st->dists, st->opacity, st->sh};
    for (int f = 0; f < 5; ++f) {
        S.p[f] = p[f];
        S.m[f] = st->exp_avg[f];
        S.v[f] = st->exp_avg_sq[f];
    }
    return S;
}

int linprim_densify_apply(int32_t type, int32_t sh_degree, int64_t n, const linprim_state* src, const float* normals,
                          const float* grad_accum, const int32_t* count, const float* max_radius,
                          const linprim_densify_params* params, const void* ws, size_t ws_bytes,
                          const linprim_state* dst, int64_t n_out, void* stream) {
    if ((type != LINPRIM_OCTAHEDRON && type != LINPRIM_TETRAHEDRON) || sh_degree < 0 || sh_degree > 3 || n < 0 ||
        n >= (int64_t(1) << 31) || n_out < 0 || n_out > 3 * n || !ws || !valid_densify(params) ||
        !state_ok(src, n) || !state_ok(dst, n_out))
        return LINPRIM_ERR_INVALID_ARG;
    if (n > 0 && (!normals || !grad_accum || !count || !max_radius)) return LINPRIM_ERR_INVALID_ARG;
    if (ws_bytes < linprim_densify_workspace_size(n)) return LINPRIM_ERR_WORKSPACE;
    if (int rc = check_device()) return rc;
    return hip_status(launch_densify_apply(type, sh_degree, n, state_set(src), normals, grad_accum, count,
                                           max_radius, densify_params(params), params->extent,
                                           (const int64_t*)ws, state_set(dst), (hipStream_t)stream));
}

int linprim_densify_noalloc(int32_t type, int32_t sh_degree, int64_t n, const linprim_state* src,
                            const float* normals, const float* grad_accum, const int32_t* count,
                            const float* max_radius, const linprim_densify_params* params, const linprim_state* dst,
                            int64_t dst_rows, int64_t* n_out, void* stream) {
    if (n > kNoAllocMaxPrims) return LINPRIM_ERR_WORKSPACE;
    if ((type != LINPRIM_OCTAHEDRON && type != LINPRIM_TETRAHEDRON) || sh_degree < 0 || sh_degree > 3 || n < 0 ||
        dst_rows < 0 || !n_out || !valid_densify(params) || !state_ok(src, n) || !state_ok(dst, dst_rows))
        return LINPRIM_ERR_INVALID_ARG;
    if (n > 0 && (!normals || !grad_accum || !count || !max_radius)) return LINPRIM_ERR_INVALID_ARG;
    if (int rc = check_device()) return rc;
    int64_t* bs = nullptr;
    if (densify_scratch(&bs) != hipSuccess) return LINPRIM_ERR_HIP;
    hipStream_t s = (hipStream_t)stream;
    // the plan writes every block sum and the total it uses: nothing to clear
    if (launch_densify_plan(type, n, src->dists, src->opacity, grad_accum, count, max_radius,
                            densify_params(params), params->extent, bs, s) != hipSuccess)
        return LINPRIM_ERR_HIP;
    const int64_t nb = (n + kDensifyItems - 1) / kDensifyItems;
    int64_t total = 0;
    if (hipMemcpyAsync(&total, bs + nb, sizeof(int64_t), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return LINPRIM_ERR_HIP;
    *n_out = total;
    if (total > dst_rows) return LINPRIM_ERR_WORKSPACE;
    return hip_status(launch_densify_apply(type, sh_degree, n, state_set(src), normals, grad_accum, count,
                                           max_radius, densify_params(params), params->extent, bs, state_set(dst),
                                           s));
}

size_t linprim_mcmc_workspace_size(int64_t n) {
    if (n < 0 || n >= (int64_t(1) << 31)) return 0;
    return mc_workspace_bytes(n);
}

int linprim_mcmc_relocate(int32_t type, int32_t sh_degree, int64_t n, const linprim_state* state,
                          const uint32_t* rand, void* ws, size_t ws_bytes, void* stream) {
    if (type != LINPRIM_OCTAHEDRON || sh_degree < 0 || sh_degree > 3 || n < 0 || n >= (int64_t(1) << 31) || !ws ||
        !state_ok(state, n) || (n > 0 && !rand))
        return LINPRIM_ERR_INVALID_ARG;
    if (ws_bytes < mc_workspace_bytes(n)) return LINPRIM_ERR_WORKSPACE;
    if (int rc = check_device()) return rc;
    return hip_status(launch_mc_relocate(n, -1, sh_degree, state_set(state), rand, (char*)ws, (hipStream_t)stream));
}

int linprim_mcmc_add(int32_t type, int32_t sh_degree, int64_t n, int64_t n_add, const linprim_state* state,
                     const uint32_t* rand, void* ws, size_t ws_bytes, void* stream) {
    if (type != LINPRIM_OCTAHEDRON || sh_degree < 0 || sh_degree > 3 || n < 0 || n_add < 0 || n_add > n ||
        n + n_add >= (int64_t(1) << 31) || !ws || !state_ok(state, n + n_add) || (n_add > 0 && !rand))
        return LINPRIM_ERR_INVALID_ARG;
    if (ws_bytes < mc_workspace_bytes(n)) return LINPRIM_ERR_WORKSPACE;
    if (int rc = check_device()) return rc;
    return hip_status(launch_mc_relocate(n, n_add, sh_degree, state_set(state), rand, (char*)ws,
                                         (hipStream_t)stream));
}

int linprim_mcmc_dead_count(const void* ws, size_t ws_bytes, int64_t n, int64_t* n_dead, void* stream) {
    if (!ws || !n_dead || n < 0 || n >= (int64_t(1) << 31)) return LINPRIM_ERR_INVALID_ARG;
    if (ws_bytes < mc_workspace_bytes(n)) return LINPRIM_ERR_WORKSPACE;
    if (n == 0) {
        *n_dead = 0;
        return LINPRIM_OK;
    }
    hipStream_t s = (hipStream_t)stream;
    int64_t v = 0;
    if (hipMemcpyAsync(&v, (const char*)ws + mc_dead_offset(n), 8, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return LINPRIM_ERR_HIP;
    *n_dead = v;
    return LINPRIM_OK;
}

int linprim_mcmc_noise(int32_t type, int64_t n, const linprim_state* state, const float* normals, float lr_means,
                       float noise_lr, void* stream) {
    if (type != LINPRIM_OCTAHEDRON || n < 0 || n >= (int64_t(1) << 31) || !state_ok(state, n) ||
        (n > 0 && !normals) || !finite_f(lr_means) || !finite_f(noise_lr))
        return LINPRIM_ERR_INVALID_ARG;
    if (int rc = check_device()) return rc;
    return hip_status(launch_mc_noise(n, state->means, state->quats, state->dists, state->opacity, normals,
                                      (double)noise_lr * (double)lr_means, (hipStream_t)stream));
}

// Loss workspace: per view, 2 floats per (channel, 32 x 32 tile) block,
// then 9 floats per pixel of the largest view.
static size_t loss_partials(const linprim_camera* cams, int32_t n_views) {
    size_t t = 0;
    for (int v = 0; v < n_views; ++v)
        t += (size_t)2 * 3 * ((cams[v].width + kLossTile - 1) / kLossTile) *
             ((cams[v].height + kLossTile - 1) / kLossTile);
    return t;
}

size_t linprim_loss_workspace_size(const linprim_camera* cams, int32_t n_views) {
    if (!valid_cams(cams, n_views)) return 0;
    size_t hw = 0;
    for (int v = 0; v < n_views; ++v) {
        const size_t x = (size_t)cams[v].width * (size_t)cams[v].height;
        if (x > hw) hw = x;
    }
    return align256(loss_partials(cams, n_views) * 4) + align256(hw * 9 * 4);
}

int linprim_loss_grad(const float* rgb, const float* target, const linprim_camera* cams, int32_t n_views,
                      float lambda, void* ws, size_t ws_bytes, float* grad, const uint32_t* skip, void* stream) {
    if (!rgb || !target || !grad || !ws || !valid_cams(cams, n_views) || !(lambda >= 0.0f && lambda <= 1.0f) ||
        grad == rgb || grad == target)
        return LINPRIM_ERR_INVALID_ARG;
    if (ws_bytes < linprim_loss_workspace_size(cams, n_views)) return LINPRIM_ERR_WORKSPACE;
    if (int rc = check_device()) return rc;
    float* partial = (float*)ws;
    float* dmaps = (float*)((char*)ws + align256(loss_partials(cams, n_views) * 4));
    int64_t px = 0;
    size_t po = 0;
    hipError_t e = hipSuccess;
    for (int v = 0; v < n_views && e == hipSuccess; ++v) {
        const int W = cams[v].width, H = cams[v].height;
        e = launch_ssim_l1(rgb + 3 * px, target + 3 * px, W, H, lambda, dmaps, partial + po, grad + 3 * px, skip,
                           (hipStream_t)stream);
        px += (int64_t)W * H;
        po += (size_t)2 * 3 * ((W + kLossTile - 1) / kLossTile) * ((H + kLossTile - 1) / kLossTile);
    }
    return hip_status(e);
}

int linprim_loss_value(const void* ws, size_t ws_bytes, const linprim_camera* cams, int32_t n_views, float lambda,
                       double* loss, void* stream) {
    if (!ws || !loss || !valid_cams(cams, n_views)) return LINPRIM_ERR_INVALID_ARG;
    if (ws_bytes < linprim_loss_workspace_size(cams, n_views)) return LINPRIM_ERR_WORKSPACE;
    const size_t np = loss_partials(cams, n_views);
    float* host = (float*)malloc(np * sizeof(float) + 1);
    if (!host) return LINPRIM_ERR_HIP;
    hipStream_t s = (hipStream_t)stream;
    if (hipMemcpyAsync(host, ws, np * sizeof(float), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) {
        free(host);
        return LINPRIM_ERR_HIP;
    }
    double total = 0.0;
    size_t po = 0;
    for (int v = 0; v < n_views; ++v) {
        const int W = cams[v].width, H = cams[v].height;
        const size_t nb = (size_t)3 * ((W + kLossTile - 1) / kLossTile) * ((H + kLossTile - 1) / kLossTile);
        double ssum = 0.0, l1 = 0.0;
        for (size_t b = 0; b < nb; ++b) {
            ssum += host[po + 2 * b];
            l1 += host[po + 2 * b + 1];
        }
        const double n = 3.0 * (double)W * (double)H;
        total += (1.0 - (double)lambda) * l1 / n + (double)lambda * (1.0 - ssum / n);
        po += 2 * nb;
    }
    free(host);
    *loss = total;
    return LINPRIM_OK;
}

int linprim_l1_grad(const float* rgb, const float* target, int64_t count, float scale, float* grad, float* partial,
                    const uint32_t* skip, void* stream) {
    if (count < 0 || (count > 0 && (!rgb || !target || !grad || !partial))) return LINPRIM_ERR_INVALID_ARG;
    return hip_status(launch_l1_grad(rgb, target, count, scale, grad, partial, skip, (hipStream_t)stream));
}

static int adam_common(const linprim_adam_group* groups, int32_t n_groups, float beta1, float beta2, float eps,
                       int32_t step, const float* bias_corr, const uint32_t* skip, void* stream) {
    if (!groups || n_groups < 1 || n_groups > 8 || (step < 1 && !bias_corr)) return LINPRIM_ERR_INVALID_ARG;
    AdamGroups G;
    memset(&G, 0, sizeof(G));
    G.count = n_groups;
    G.block0[0] = 0;
    const int64_t per_block = 256 * 4;
    auto aligned = [](const void* p) { return ((uintptr_t)p & 15u) == 0; };
    for (int k = 0; k < n_groups; ++k) {
        const linprim_adam_group& g = groups[k];
        if (g.numel < 0 || (g.numel > 0 && (!g.param || !g.grad || !g.exp_avg || !g.exp_avg_sq)))
            return LINPRIM_ERR_INVALID_ARG;
        if (g.period < 0 || (g.period > 0 && (g.head < 0 || g.head > g.period))) return LINPRIM_ERR_INVALID_ARG;
        G.param[k] = g.param;
        G.grad[k] = g.grad;
        G.m[k] = g.exp_avg;
        G.v[k] = g.exp_avg_sq;
        G.numel[k] = g.numel;
        G.lr[k] = g.lr;
        G.lr_tail[k] = g.lr_tail;
        G.period[k] = g.period;
        G.head[k] = g.head;
        G.lo[k] = g.lo;
        G.hi[k] = g.hi;
        G.vec[k] = aligned(g.param) && aligned(g.grad) && aligned(g.exp_avg) && aligned(g.exp_avg_sq);
        G.block0[k + 1] = G.block0[k] + (g.numel + per_block - 1) / per_block;
    }
    if (G.block0[n_groups] > 0x7fffffffLL) return LINPRIM_ERR_INVALID_ARG;
    const double bc1 = bias_corr ? 1.0 : 1.0 - pow((double)beta1, (double)step);
    const double bc2 = bias_corr ? 1.0 : 1.0 - pow((double)beta2, (double)step);
    return hip_status(launch_adam(G, beta1, beta2, eps, (float)bc1, (float)bc2, bias_corr, skip,
                                  (hipStream_t)stream));
}

int linprim_adam_step(const linprim_adam_group* groups, int32_t n_groups, float beta1, float beta2, float eps,
                      int32_t step, void* stream) {
    return adam_common(groups, n_groups, beta1, beta2, eps, step, nullptr, nullptr, stream);
}

int linprim_adam_step_dev(const linprim_adam_group* groups, int32_t n_groups, float beta1, float beta2, float eps,
                          const float* bias_corr, const uint32_t* skip, void* stream) {
    if (!bias_corr) return LINPRIM_ERR_INVALID_ARG;
    return adam_common(groups, n_groups, beta1, beta2, eps, 0, bias_corr, skip, stream);
}

int linprim_step_guard(const linprim_prims* prims, const linprim_camera* cams, int32_t n_views,
                       const linprim_tuning* tuning, const void* view_ws, size_t view_ws_bytes, uint32_t* guard,
                       void* stream) {
    if (!prims || !guard || !view_ws || !valid_cams(cams, n_views) || !valid_tuning(tuning))
        return LINPRIM_ERR_INVALID_ARG;
    const ViewLayout L = view_layout(prims->n, cams, n_views, tile_of(tuning));
    if (view_ws_bytes < L.total) return LINPRIM_ERR_WORKSPACE;
    if (int rc = check_device()) return rc;
    return hip_status(launch_step_guard(view_ws, L, guard, (hipStream_t)stream));
}

int linprim_read_status(const void* view_ws, int64_t* pairs_needed, int32_t* overflow, void* stream) {
    if (!view_ws || !pairs_needed || !overflow) return LINPRIM_ERR_INVALID_ARG;
    Status st;
    hipStream_t s = (hipStream_t)stream;
    if (hipMemcpyAsync(&st, view_ws, sizeof(Status), hipMemcpyDeviceToHost, s) != hipSuccess) return LINPRIM_ERR_HIP;
    if (hipStreamSynchronize(s) != hipSuccess) return LINPRIM_ERR_HIP;
    *pairs_needed = (int64_t)st.n_pairs;
    *overflow = (int32_t)st.overflow;
    return LINPRIM_OK;
}

const char* linprim_strerror(int code) {
    switch (code) {
        case LINPRIM_OK: return "ok";
        case LINPRIM_ERR_INVALID_ARG: return "invalid argument";
        case LINPRIM_ERR_WORKSPACE: return "workspace too small";
        case LINPRIM_ERR_PAIR_OVERFLOW: return "more (tile, primitive) pairs than the pair workspace holds";
        case LINPRIM_ERR_HIP: return "HIP runtime error";
        case LINPRIM_ERR_DEVICE: return "unsupported device (gfx950 required)";
        default: return "unknown error";
    }
}

int linprim_debug_pointers(const linprim_prims* prims, const linprim_camera* cams, int32_t n_views,
                           const linprim_tuning* tuning, const void* view_ws, const void* pair_ws, int64_t max_pairs,
                           void** payload, void** depth_keys, void** tiles_touched, void** offsets, void** keys,
                           void** values, void** ranges, void** order_fwd, void** order_bwd) {
    if (!view_ws || !pair_ws) return LINPRIM_ERR_INVALID_ARG;
    ViewLayout L;
    PairLayout P;
    if (int rc = prepare(prims, cams, n_views, tuning, (size_t)-1, (size_t)-1, max_pairs, L, P)) return rc;
    const char* v = (const char*)view_ws;
    const char* p = (const char*)pair_ws;
    const int in_b = result_buffer(L, tuning);
    if (payload) *payload = (void*)(v + L.payload);
    if (depth_keys) *depth_keys = (void*)(v + L.depth_keys);
    if (tiles_touched) *tiles_touched = (void*)(v + L.tiles);
    if (offsets) *offsets = (void*)(v + L.offsets);
    if (keys) *keys = (void*)(p + (in_b ? P.keys_b : P.keys_a));
    if (values) *values = (void*)(p + (in_b ? P.vals_b : P.vals_a));
    if (ranges) *ranges = (void*)(v + L.ranges);
    if (order_fwd) *order_fwd = (void*)(v + L.order);
    if (order_bwd) *order_bwd = (void*)(v + L.order_bwd);
    return LINPRIM_OK;
}

}  // extern "C"
