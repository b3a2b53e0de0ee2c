// linprim_common.h -- internal layout and device helpers of the gfx950
// rasterizer for transparent octahedra and tetrahedra (LinPrim, arXiv
// 2501.16312).  Included by every kernel file of liblinprim.so.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/linprim.h"

namespace linprim {

// ----------------------------------------------------------------------------
// Constants.
// ----------------------------------------------------------------------------
constexpr float kAlphaScale = 0.99f;      // Eq. 1
constexpr double kAlphaScaleD = 0.99;
constexpr float kTStop = 1e-3f;           // cumulative opacity 0.999 (Sec. 3.2)
constexpr float kOMax = 0.99f;            // opacity clamp: 1 - o >= 0.01
constexpr float kOneMinusOMax = 0.01f;
constexpr double kInvSqrt3 = 0.57735026918962576451;
constexpr double kLog2e = 1.44269504088896340736;
constexpr int kMaxViews = 4096;
constexpr int kRecordWords = 32;          // payload record: 32 x 4 bytes
constexpr int kGradWords = 20;            // backward record per (tile, primitive) pair and 8x8 group

// ----------------------------------------------------------------------------
// Payload record of one (view, primitive), 32 dwords, written by the
// preprocess kernel and read with scalar loads by the render kernels.
//   [0..3]  int   pixel rectangle i0, j0, i1, j1 (inclusive); i0 = -1 if culled
//   [4]     float sigma * log2(e)            (so exp(-sigma d) = exp2(-s2 d))
//   [5..7]  float rgb
//   [8..11] float the rectangle's centre (i0 + i1)/2, (j0 + j1)/2 and
//           half-extents (i1 - i0)/2, (j1 - j0)/2 (half-integers, exact)
//   octahedron:
//   [12..27] float 4 slabs x (A, B, Dup, Dlo): with ki = i - (i0 + i1)/2,
//            kj = j - (j0 + j1)/2 the slab is
//            A ki + B kj + Dlo <= z' <= A ki + B kj + Dup
//   tetrahedron:
//   [12..20] float 3 upper planes (A, B, D): z' <= A ki + B kj + D
//   [21..29] float 3 lower planes (A, B, D): z' >= A ki + B kj + D
//   [31]     int   face of each of the 6 plane slots, 2 bits each
//   [30]    float sigma
// The chord through the primitive at a pixel is
//   max(0, min over upper planes - max over lower planes).
//
// Exact variant (no ray space), both types: the pixel ray is
// X(tau) = z_c (1 + tau) D with D = ((i + 1/2 - cx)/fx, (j + 1/2 - cy)/fy, 1)
// and z_c the centre's camera depth.  Plane k of the camera-space primitive,
// n_k . (X - centre) = h, crosses it at tau = (u_k + h) / (c_k - u_k) with
//   u_k = a_k ki + b_k kj + g_k  (= n_k . (centre - z_c D)),  c_k = n_k . centre.
//   [12 + 4 k .. 15 + 4 k]  float a_k, b_k, g_k, c_k   (k = 0..3)
//   octahedron: slab k is -1 <= n_k . (X - centre) <= 1 (both signs of h);
//   tetrahedron: face k is n_k . (X - centre) <= 1, an exit where
//   c_k - u_k >= 0 and an entry elsewhere;
//   [4]  float sigma z_c log2(e),  [30] float sigma z_c.
// The chord is |D| z_c (min exits - max entries), so that
// exp(-sigma chord) = exp2(-[4] |D| (min exits - max entries)).
// ----------------------------------------------------------------------------
enum : int {
    R_I0 = 0, R_J0 = 1, R_I1 = 2, R_J1 = 3, R_S2 = 4, R_RGB = 5, R_FI0 = 8, R_FJ0 = 9, R_FWI = 10,
    R_FWJ = 11, R_PLANES = 12, R_SIGMA = 30, R_FACEMAP = 31
};

// Per-view constants, in the view table at the front of the view workspace.
struct ViewInfo {
    double Rw[9];
    double tw[3];
    double cam_pos[3];
    double fx, fy, cx, cy, near_z;
    int32_t width, height, tiles_x, tiles_y;
    int64_t tile_base;   // first global tile id of this view
    int64_t pix_base;    // first pixel of this view in the packed outputs
    int32_t pad[4];
};

// Header of the view workspace.
struct Status {
    uint64_t n_pairs;      // written by the scan
    uint32_t overflow;     // set by bin_sort when n_pairs > capacity
    uint32_t n_big;        // slots with more than kBigRun records, up to kHugeRun tiles (list in ViewLayout::big)
    uint64_t capacity;
    uint32_t n_long;       // tiles whose list is sorted by the long-list kernel
    uint32_t n_vis;        // (view, primitive) slots that touch a tile (list in ViewLayout::vis)
    uint32_t n_huge;       // slots with more than kHugeRun tiles (list in ViewLayout::huge)
    uint32_t n_mid;        // slots with kMidRun < records <= kBigRun (listed from the end of ViewLayout::big)
    uint64_t pad[3];
};

// Offsets into the view workspace (all 256-byte aligned).
struct ViewLayout {
    size_t status, views, payload, depth_keys, tiles, offsets, block_sums, ranges, big, long_list, vis, stats, order,
        order_bwd, order_sums, huge, trect, total;
    int64_t n, n_views, n_tiles_total, scan_blocks;
};

// Offsets into the pair workspace.
struct PairLayout {
    size_t keys_a, keys_b, vals_a, vals_b, hist, grads, total;
    int64_t capacity, sort_blocks;
};

constexpr int kScanItems = 4096;     // elements per scan block (256 threads x 16)
// Up to this many scan blocks, each block adds the totals of the blocks
// before it itself (8192 blocks: 32M slots); beyond, a single block turns
// the totals into prefixes first.
constexpr int64_t kScanDirectBlocks = 8192;
// Tiles per block of the render order kernels (256 threads x 4), and the
// same choice for their per-block counts (256 blocks: 256K tiles).
constexpr int64_t kOrderDirectBlocks = 256;
// Tiles per block of the render-order kernels: 256, or a multiple of 256 (at
// most 4096) so that up to 16M tiles need no more than kOrderDirectBlocks
// blocks, whose counts every block then adds itself (no separate prefix).
__host__ __device__ inline int order_items(int64_t n_tiles) {
    const int64_t per = 256 * kOrderDirectBlocks;
    int64_t rounds = (n_tiles + per - 1) / per;
    rounds = rounds < 1 ? 1 : (rounds > 16 ? 16 : rounds);
    return (int)(256 * rounds);
}
constexpr int kSortThreads = 256;
constexpr int kSortItems = 4;        // keys per thread per sort block
constexpr int kSortTile = kSortThreads * kSortItems;

inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

ViewLayout view_layout(int64_t n, const linprim_camera* cams, int32_t n_views, int tile);
PairLayout pair_layout(int64_t max_pairs, int digit_bits, int tile);
int key_tile_bits(int64_t n_tiles_total);

// ----------------------------------------------------------------------------
// Host-side launchers (one per kernel file).
// ----------------------------------------------------------------------------
// Inclusive prefix sum over the 64 lanes of a wave by DPP steps (every lane
// must be active): row shifts by 1, 2, 4 and 8 within each row of 16 lanes,
// then the last lane of row 0 added to row 1 and of row 2 to row 3, then lane
// 31 to rows 2 and 3.
__device__ inline uint32_t wave_incl_scan_u32(uint32_t v) {
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xF, 0xF, true);    // row_shr:1
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xF, 0xF, true);    // row_shr:2
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xF, 0xF, true);    // row_shr:4
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xF, 0xF, true);    // row_shr:8
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xA, 0xF, false);   // row_bcast:15
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xC, 0xF, false);   // row_bcast:31
    return v;
}

// Views passed by value in one launch argument.
constexpr int kViewChunk = 8;
struct ViewChunk {
    ViewInfo v[kViewChunk];
};
hipError_t launch_store_views(const linprim_camera* cams, int32_t n_views, int tile, ViewInfo* views,
                              hipStream_t stream);
// cams: the cameras, when the views are not yet stored in the workspace
hipError_t launch_preprocess(const linprim_prims& p, int32_t n_views, int tile, bool exact, bool aa,
                             const ViewLayout& L, char* ws, hipStream_t stream, const linprim_camera* cams);
hipError_t launch_scan(const ViewLayout& L, char* ws, int tile, hipStream_t stream);

// A (view, primitive) slot whose gradient records number more than kBigRun
// has them summed in kBigChunks chunks, each chunk's sum written into the
// chunk's first record: by one wave, four lanes per chunk, if the slot is on
// the scan's big list (up to kHugeRun tiles), else (more than kHugeRun tiles:
// the huge list) by kBigChunks waves, one per chunk.  A slot with more than
// kMidRun records, up to kBigRun, is summed in record order by twenty lanes,
// one word each, into its first record (the mid list, stored from the end of
// the big list's array: each slot is on at most one of the two).  The thread
// of a slot with at most kMidRun records sums them itself.
constexpr int kBigRun = 64;
constexpr int kMidRun = 8;
// Slots whose tile rectangle holds more than kHugeRun tiles have their pairs
// emitted by every wave of the emission grid together.
constexpr int kHugeRun = 1024;

// Tile rectangle of a visible slot, packed for the emission kernel (tile
// coordinates are below 2^16): x = tx0 | ty0 << 16, y = ntx | nty << 16.
__host__ __device__ inline uint2 pack_tile_rect(int i0, int j0, int i1, int j1, int tile_shift) {
    const int tx0 = i0 >> tile_shift, ty0 = j0 >> tile_shift;
    const int ntx = (i1 >> tile_shift) - tx0 + 1, nty = (j1 >> tile_shift) - ty0 + 1;
    return make_uint2((uint32_t)tx0 | ((uint32_t)ty0 << 16), (uint32_t)ntx | ((uint32_t)nty << 16));
}

// The render kernels take the tiles in the orders written by bin_sort.  The
// backward's: by list length, longest first, in classes of lengths (> 192,
// > 128, ..., > 4, > 0, empty), each class in tile order, so that the longest
// walks start first and the waves that start last are short (the exact
// variant's forward takes it too).  The ray-space forward's:
// groups of consecutive classes (the last class of each group in
// kFwdGroupLast), each group in tile order.
constexpr int kOrderClasses = 16;
__device__ constexpr uint32_t kOrderBounds[kOrderClasses - 1] = {192, 128, 96, 72, 56, 48, 40, 32,
                                                                 26, 20, 16, 12, 8, 4, 0};
constexpr int kFwdGroups = 3;   // lists of more than 128 pairs, of 73-128, the others
__device__ constexpr int kFwdGroupLast[kFwdGroups] = {1, 3, 15};
constexpr int kBigChunks = 16;
__host__ __device__ inline int big_chunk_start(int c, int nrec) {
    return (int)(((int64_t)c * nrec) / kBigChunks);
}
// Pairs are sorted per tile (count, scan, scatter, per-list sort) unless
// `radix` selects the global LSD radix sort of the full keys.
// Which pair buffer (0: a, 1: b) holds the sorted pairs after bin_sort.
int sorted_buffer(int64_t n_tiles_total, bool radix, int digit_bits);
hipError_t launch_bin_sort(const ViewLayout& L, char* vws, const PairLayout& P, char* pws, bool radix,
                           int tile, int digit_bits, int32_t n_views, const linprim_camera* cams,
                           hipStream_t stream, int* result_in_b);
hipError_t launch_render_fwd(const ViewLayout& L, const char* vws, const PairLayout& P, const char* pws,
                             int result_in_b, int type, bool exact, int tile, int32_t n_views, const float bg[3],
                             float* out_rgb, float* out_T, int32_t* out_last, hipStream_t stream);
hipError_t launch_render_bwd(const ViewLayout& L, const char* vws, const PairLayout& P, char* pws,
                             int result_in_b, int type, bool exact, int tile, int32_t n_views, const float bg[3],
                             const float* out_T, const int32_t* out_last, const float* grad_rgb,
                             hipStream_t stream);
hipError_t launch_preprocess_bwd(const linprim_prims& p, int32_t n_views, int tile, bool exact, bool aa,
                                 const ViewLayout& L,
                                 const char* vws, const PairLayout& P, const char* pws, float* g_means,
                                 float* g_quats, float* g_dists, float* g_opacity, float* g_sh,
                                 hipStream_t stream);

struct AdamGroups {
    float* param[8];
    const float* grad[8];
    float* m[8];
    float* v[8];
    int64_t numel[8];
    int64_t block0[9];    // first block of each group (prefix of per-group block counts)
    float lr[8];
    float lr_tail[8];     // learning rate of positions (i mod period) >= head
    int period[8], head[8];
    float lo[8], hi[8];   // projection box after the update
    int vec[8];           // all four arrays 16-byte aligned
    int count;
};
// Adaptive population control (Sec. 3.4; thresholds of App. G).
struct DensifyParams {
    float grad_threshold, min_opacity, max_size_frac, max_radius, clone_size_frac, shrink;
};
struct StateSet {
    float* p[5];     // means, quats, dists, opacity, sh
    float* m[5];     // Adam first moments (all null: none)
    float* v[5];     // Adam second moments
};
constexpr int kDensifyItems = 1024;   // primitives per scan block
constexpr int64_t kNoAllocMaxPrims = LINPRIM_NOALLOC_MAX_PRIMS;
static_assert(kNoAllocMaxPrims % kDensifyItems == 0, "whole scan blocks");
// Per-device address of the static scratch of linprim_densify_noalloc.
hipError_t densify_scratch(int64_t** out);
hipError_t launch_accumulate_stats(int64_t n, int32_t n_views, const ViewLayout& L, const char* vws,
                                   float* grad_accum, int32_t* count, float* max_radius, hipStream_t s);
hipError_t launch_densify_plan(int type, int64_t n, const float* dists, const float* opacity,
                               const float* grad_accum, const int32_t* count, const float* max_radius,
                               const DensifyParams& dp, float extent, int64_t* block_sums, hipStream_t s);
hipError_t launch_densify_apply(int type, int sh_degree, int64_t n, const StateSet& src, const float* normals,
                                const float* grad_accum, const int32_t* count, const float* max_radius,
                                const DensifyParams& dp, float extent, const int64_t* block_sums,
                                const StateSet& dst, hipStream_t s);

// LinPrim-MCMC population steps (Sec. 3.4), octahedra.
size_t mc_workspace_bytes(int64_t n);
int64_t mc_dead_offset(int64_t n);
hipError_t launch_mc_relocate(int64_t n, int64_t n_add, int sh_degree, const StateSet& S, const uint32_t* rnd,
                              char* ws, hipStream_t s);
hipError_t launch_mc_noise(int64_t n, float* means, const float* quats, const float* dists, const float* opacity,
                           const float* eps, double scale, hipStream_t s);

// Photometric loss (Sec. 3.4 "Optimization"), one view [3, H, W].
constexpr int kLossTile = 32;
hipError_t launch_ssim_l1(const float* rgb, const float* target, int W, int H, float lam, float* dmaps,
                          float* partial, float* grad, const uint32_t* skip, hipStream_t s);

hipError_t launch_adam(const AdamGroups& G, float beta1, float beta2, float eps, float bc1, float bc2,
                       const float* bias_corr, const uint32_t* skip, hipStream_t s);
hipError_t launch_l1_grad(const float* rgb, const float* target, int64_t count, float scale, float* grad,
                          float* partial, const uint32_t* skip, hipStream_t s);
hipError_t launch_step_guard(const void* view_ws, const ViewLayout& L, uint32_t* guard, hipStream_t s);

// ----------------------------------------------------------------------------
// Device helpers.
// ----------------------------------------------------------------------------

template <int CTRL, int ROW_MASK = 0xF>
__device__ inline float dpp_mov(float src) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(src), CTRL, ROW_MASK, 0xF, false));
}

// Sums 20 values over the 64 lanes of a wave and leaves each total in one
// lane: two cross-half swaps (permlane32 / permlane16) pair the values so
// that every 16-lane row holds 5 of them, then four DPP steps inside the
// row each halve the values a lane keeps while doubling the set of lanes
// they are summed over (row mirror: lane i with 15 - i; half-row mirror:
// i with 7 - i; quad swaps: i with i ^ 2, then i with i ^ 1).  Lane L of row
// r = L / 16 ends with the total of value v + 5 r, v = 4 b1 + 2 b2 + b3 from
// the bits b1, b2, b3 of L; lanes with v >= 5, and the odd lane of each pair
// that holds a duplicate, do not write (see reduce20_index).
__device__ inline float wave_reduce20(const float (&v)[20], int lane) {
    float a[10];
#pragma unroll
    for (int j = 0; j < 10; ++j) {
        const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(v[j]), __float_as_uint(v[j + 10]), false, false);
        a[j] = __uint_as_float(r[0]) + __uint_as_float(r[1]);
    }
    float b[6];
#pragma unroll
    for (int j = 0; j < 5; ++j) {
        const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(a[j]), __float_as_uint(a[j + 5]), false, false);
        b[j] = __uint_as_float(r[0]) + __uint_as_float(r[1]);
    }
    b[5] = 0.0f;
    const bool h3 = (lane >> 3) & 1, h2 = (lane >> 2) & 1, h1 = (lane >> 1) & 1;
    float c[4];
#pragma unroll
    for (int p = 0; p < 3; ++p) {                       // lanes i and 15 - i
        const float keep = h3 ? b[2 * p + 1] : b[2 * p];
        const float give = h3 ? b[2 * p] : b[2 * p + 1];
        c[p] = keep + dpp_mov<0x140>(give);
    }
    c[3] = 0.0f;
    float d[2];
#pragma unroll
    for (int q = 0; q < 2; ++q) {                       // lanes i and 7 - i of a half row
        const float keep = h2 ? c[2 * q + 1] : c[2 * q];
        const float give = h2 ? c[2 * q] : c[2 * q + 1];
        d[q] = keep + dpp_mov<0x141>(give);
    }
    const float keep = h1 ? d[1] : d[0];               // lanes i and i ^ 2
    const float give = h1 ? d[0] : d[1];
    float e = keep + dpp_mov<0x4E>(give);
    e += dpp_mov<0xB1>(e);                              // lanes i and i ^ 1
    return e;
}

// Which of the 20 totals lane L writes after wave_reduce20 (-1: none).
__device__ inline int reduce20_index(int lane) {
    const int i = lane & 15;
    const int v = 4 * ((i >> 1) & 1) + 2 * ((i >> 2) & 1) + ((i >> 3) & 1);
    return ((i & 1) == 0 && v < 5) ? v + 5 * (lane >> 4) : -1;
}

// Rotation of q / |q| written with s = 2 / |q|^2 (no square root).  The
// expressions and their left-to-right order are part of the binning
// contract: compiled without contraction into fused multiply-adds.
#pragma clang fp contract(off)
__device__ inline bool quat_rotation_d(double w, double x, double y, double z, double R[9]) {
    const double n2 = w * w + x * x + y * y + z * z;
    if (!(n2 > 0.0) || !isfinite(n2)) return false;
    const double s = 2.0 / n2;
    R[0] = 1.0 - s * (y * y + z * z);
    R[1] = s * (x * y - w * z);
    R[2] = s * (x * z + w * y);
    R[3] = s * (x * y + w * z);
    R[4] = 1.0 - s * (x * x + z * z);
    R[5] = s * (y * z - w * x);
    R[6] = s * (x * z - w * y);
    R[7] = s * (y * z + w * x);
    R[8] = 1.0 - s * (x * x + y * y);
    return true;
}

// Tetrahedron corner directions, before the 1/sqrt(3) scale.
__device__ constexpr double kTetDir[4][3] = {{1, 1, 1}, {1, -1, -1}, {-1, 1, -1}, {-1, -1, 1}};

// Geometry of one primitive in one view, in double precision.
struct Geom {
    double R[9];        // primitive rotation
    double o[4][3];     // world-space offsets of the axes / corners
    double oc[4][3];    // camera-space offsets
    double tc[3];       // camera-space centre
    double c[3];        // ray-space centre
    double a[4][3];     // ray-space offsets
    double J[9];        // ray-space Jacobian at tc (row-major)
    int rect[4];
    uint32_t key;
    double radius;      // half the larger side of the projected bounding box (pixels)
};

// Builds the primitive, transforms it and bounds it.  Returns false if the
// primitive is culled.  The rectangle and key computations follow the
// binning contract exactly (double precision, fixed order, no contraction).
// The 2D anti-aliasing filter (appendix "Anti-Aliasing"; filter size 0.1
// pixel, App. G): the ray-space corners on the tiling box move outward,
// parallel to the screen, so that the box grows by the filter size per
// axis: an octahedron's axis vector carries two mirrored corners and moves
// by half of it, and a tetrahedron's extreme corners move by half of it
// each.  All corners that attain an extreme move.  The shift is a constant,
// so gradients with respect to the offsets pass through unchanged.
constexpr double kAaSize = 0.1;

__device__ inline void antialias_shift(int type, double a[4][3]) {
#pragma unroll
    for (int ax = 0; ax < 2; ++ax) {
        if (type == LINPRIM_OCTAHEDRON) {
            double ext = 0.0;
#pragma unroll
            for (int k = 0; k < 3; ++k)
                if (fabs(a[k][ax]) > ext) ext = fabs(a[k][ax]);
            double sh[3];
#pragma unroll
            for (int k = 0; k < 3; ++k) sh[k] = (fabs(a[k][ax]) == ext) ? copysign(0.5 * kAaSize, a[k][ax]) : 0.0;
#pragma unroll
            for (int k = 0; k < 3; ++k) a[k][ax] += sh[k];
        } else {
            double lo = a[0][ax], hi = a[0][ax];
#pragma unroll
            for (int i = 1; i < 4; ++i) {
                if (a[i][ax] < lo) lo = a[i][ax];
                if (a[i][ax] > hi) hi = a[i][ax];
            }
            double sh[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                sh[i] = 0.0;
                if (a[i][ax] == lo) sh[i] -= 0.5 * kAaSize;
                if (a[i][ax] == hi) sh[i] += 0.5 * kAaSize;
            }
#pragma unroll
            for (int i = 0; i < 4; ++i) a[i][ax] += sh[i];
        }
    }
}

// The view-independent part of build_geometry: rotation, world-space
// offsets, validity of the inputs.  Returns false for a primitive no view
// can see (degenerate rotation, non-positive or non-finite distances,
// non-finite centre, opacity outside [0, 1]).
__device__ inline bool build_world(int type, const float* mu_f, const float* q_f, const float* d_f, float alpha,
                                   Geom& G) {
    const int na = (type == LINPRIM_OCTAHEDRON) ? 3 : 4;
    if (!quat_rotation_d((double)q_f[0], (double)q_f[1], (double)q_f[2], (double)q_f[3], G.R)) return false;
    double d[4];
    for (int k = 0; k < na; ++k) {
        d[k] = (double)d_f[k];
        if (!(d[k] > 0.0) || !isfinite(d[k])) return false;
    }
    const double mu[3] = {(double)mu_f[0], (double)mu_f[1], (double)mu_f[2]};
    if (!isfinite(mu[0]) || !isfinite(mu[1]) || !isfinite(mu[2])) return false;
    const double al = (double)alpha;
    if (!(al >= 0.0 && al <= 1.0)) return false;
    if (type == LINPRIM_OCTAHEDRON) {
        for (int k = 0; k < 3; ++k)
            for (int r = 0; r < 3; ++r) G.o[k][r] = G.R[3 * r + k] * d[k];
    } else {
        for (int i = 0; i < 4; ++i) {
            const double g = d[i] * kInvSqrt3;
            for (int r = 0; r < 3; ++r)
                G.o[i][r] = (kTetDir[i][0] * G.R[3 * r + 0] + kTetDir[i][1] * G.R[3 * r + 1] +
                             kTetDir[i][2] * G.R[3 * r + 2]) * g;
        }
    }
    return true;
}

// The per-view part: G.R and G.o from build_world; the rest of G from the
// camera.  Returns false if the primitive is culled in this view.
__device__ inline bool build_view(int type, bool exact, bool aa, const float* mu_f, const ViewInfo& V, Geom& G) {
    const int na = (type == LINPRIM_OCTAHEDRON) ? 3 : 4;
    const double mu[3] = {(double)mu_f[0], (double)mu_f[1], (double)mu_f[2]};
    for (int r = 0; r < 3; ++r)
        G.tc[r] = V.Rw[3 * r + 0] * mu[0] + V.Rw[3 * r + 1] * mu[1] + V.Rw[3 * r + 2] * mu[2] + V.tw[r];
    if (!(G.tc[2] > V.near_z)) return false;
    for (int k = 0; k < na; ++k)
        for (int r = 0; r < 3; ++r)
            G.oc[k][r] = V.Rw[3 * r + 0] * G.o[k][0] + V.Rw[3 * r + 1] * G.o[k][1] + V.Rw[3 * r + 2] * G.o[k][2];

    const double iz = 1.0 / G.tc[2];
    const double px = V.fx * G.tc[0] * iz, py = V.fy * G.tc[1] * iz;
    const double cxp = px + V.cx, cyp = py + V.cy;
    const double J00 = V.fx * iz, J02 = -(px * iz), J11 = V.fy * iz, J12 = -(py * iz);
    const double l = sqrt(G.tc[0] * G.tc[0] + G.tc[1] * G.tc[1] + G.tc[2] * G.tc[2]);
    G.J[0] = J00; G.J[1] = 0.0; G.J[2] = J02;
    G.J[3] = 0.0; G.J[4] = J11; G.J[5] = J12;
    G.J[6] = G.tc[0] / l; G.J[7] = G.tc[1] / l; G.J[8] = G.tc[2] / l;
    G.c[0] = cxp; G.c[1] = cyp; G.c[2] = l;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        if (k >= na) break;
        G.a[k][0] = J00 * G.oc[k][0] + J02 * G.oc[k][2];
        G.a[k][1] = J11 * G.oc[k][1] + J12 * G.oc[k][2];
        G.a[k][2] = G.J[6] * G.oc[k][0] + G.J[7] * G.oc[k][1] + G.J[8] * G.oc[k][2];
    }
    if (aa) antialias_shift(type, G.a);
    double xmin = INFINITY, xmax = -INFINITY, ymin = INFINITY, ymax = -INFINITY;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        if (k >= na) break;
        const double ax = G.a[k][0], ay = G.a[k][1];
        const double xp = cxp + ax, yp = cyp + ay;
        if (xp < xmin) xmin = xp;
        if (xp > xmax) xmax = xp;
        if (yp < ymin) ymin = yp;
        if (yp > ymax) ymax = yp;
        if (type == LINPRIM_OCTAHEDRON) {
            const double xm = cxp - ax, ym = cyp - ay;
            if (xm < xmin) xmin = xm;
            if (xm > xmax) xmax = xm;
            if (ym < ymin) ymin = ym;
            if (ym > ymax) ymax = ym;
        }
    }
    if (exact) {
        // without ray space the footprint is bounded by the perspective
        // projections of the corners; a corner at or in front of the near
        // plane has none, and the primitive is culled
        xmin = INFINITY; xmax = -INFINITY; ymin = INFINITY; ymax = -INFINITY;
        const int nc = (type == LINPRIM_OCTAHEDRON) ? 6 : 4;
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            if (k >= nc) break;
            double v[3];
#pragma unroll
            for (int r = 0; r < 3; ++r) {
                if (type == LINPRIM_OCTAHEDRON)
                    v[r] = (k & 1) ? G.tc[r] - G.oc[k >> 1][r] : G.tc[r] + G.oc[k >> 1][r];
                else
                    v[r] = G.tc[r] + G.oc[k][r];
            }
            if (!(v[2] > V.near_z)) return false;
            const double xp = V.fx * v[0] / v[2] + V.cx;
            const double yp = V.fy * v[1] / v[2] + V.cy;
            if (xp < xmin) xmin = xp;
            if (xp > xmax) xmax = xp;
            if (yp < ymin) ymin = yp;
            if (yp > ymax) ymax = yp;
        }
    }
    if (!isfinite(xmin) || !isfinite(xmax) || !isfinite(ymin) || !isfinite(ymax)) return false;
    G.radius = 0.5 * fmax(xmax - xmin, ymax - ymin);
    double fi0 = ceil(xmin - 0.5), fi1 = floor(xmax - 0.5);
    double fj0 = ceil(ymin - 0.5), fj1 = floor(ymax - 0.5);
    if (fi0 < 0.0) fi0 = 0.0;
    if (fj0 < 0.0) fj0 = 0.0;
    if (fi1 > (double)(V.width - 1)) fi1 = (double)(V.width - 1);
    if (fj1 > (double)(V.height - 1)) fj1 = (double)(V.height - 1);
    if (fi0 > fi1 || fj0 > fj1) return false;
    G.rect[0] = (int)fi0; G.rect[1] = (int)fj0; G.rect[2] = (int)fi1; G.rect[3] = (int)fj1;
    const float zf = (float)G.tc[2];
    G.key = __float_as_uint(zf);
    return true;
}

__device__ inline bool build_geometry(int type, bool exact, bool aa, const float* mu_f, const float* q_f,
                                      const float* d_f, float alpha, const ViewInfo& V, Geom& G) {
    return build_world(type, mu_f, q_f, d_f, alpha, G) && build_view(type, exact, aa, mu_f, V, G);
}
#pragma clang fp contract(on)

// Real SH basis, degree <= 3, Condon-Shortley phase for odd m, ordered
// l = 0..3, m = -l..l; constants from their closed forms.
struct ShConst {
    double c0, c1, c2a, c2b, c2c, c3a, c3b, c3c, c3d, c3e;
};

__device__ inline ShConst sh_constants() {
    const double pi = 3.14159265358979323846;
    ShConst K;
    K.c0 = 0.5 * sqrt(1.0 / pi);
    K.c1 = sqrt(3.0 / (4.0 * pi));
    K.c2a = 0.5 * sqrt(15.0 / pi);
    K.c2b = 0.25 * sqrt(5.0 / pi);
    K.c2c = 0.25 * sqrt(15.0 / pi);
    K.c3a = 0.25 * sqrt(35.0 / (2.0 * pi));
    K.c3b = 0.5 * sqrt(105.0 / pi);
    K.c3c = 0.25 * sqrt(21.0 / (2.0 * pi));
    K.c3d = 0.25 * sqrt(7.0 / pi);
    K.c3e = 0.25 * sqrt(105.0 / pi);
    return K;
}

// The basis in single precision, degree fixed at compile time (the colour
// only needs float accuracy; the constants are computed in double from
// their closed forms and rounded once).
template <int DEG>
__device__ inline void sh_eval_f(float x, float y, float z, float Y[16]) {
    const ShConst K = sh_constants();
    const float c0 = (float)K.c0, c1 = (float)K.c1, c2a = (float)K.c2a, c2b = (float)K.c2b, c2c = (float)K.c2c;
    const float c3a = (float)K.c3a, c3b = (float)K.c3b, c3c = (float)K.c3c, c3d = (float)K.c3d, c3e = (float)K.c3e;
    Y[0] = c0;
    if (DEG >= 1) {
        Y[1] = -c1 * y;
        Y[2] = c1 * z;
        Y[3] = -c1 * x;
    }
    if (DEG >= 2) {
        const float xx = x * x, yy = y * y, zz = z * z;
        Y[4] = c2a * x * y;
        Y[5] = -c2a * y * z;
        Y[6] = c2b * (2.0f * zz - xx - yy);
        Y[7] = -c2a * x * z;
        Y[8] = c2c * (xx - yy);
        if (DEG >= 3) {
            Y[9] = -c3a * y * (3.0f * xx - yy);
            Y[10] = c3b * x * y * z;
            Y[11] = -c3c * y * (4.0f * zz - xx - yy);
            Y[12] = c3d * z * (2.0f * zz - 3.0f * xx - 3.0f * yy);
            Y[13] = -c3c * x * (4.0f * zz - xx - yy);
            Y[14] = c3e * z * (xx - yy);
            Y[15] = -c3a * x * (xx - 3.0f * yy);
        }
    }
}


// Loads the (DEG+1)^2 x 3 SH coefficients of one primitive into registers,
// every load issued before the first use (16-byte loads for degree 3).
template <int DEG>
__device__ inline void load_sh(const float* __restrict__ p, float out[48]) {
    constexpr int NF = 3 * (DEG + 1) * (DEG + 1);
    if (NF % 4 == 0) {
        const float4* p4 = reinterpret_cast<const float4*>(p);
#pragma unroll
        for (int k = 0; k < NF / 4; ++k) {
            const float4 x = p4[k];
            out[4 * k] = x.x;
            out[4 * k + 1] = x.y;
            out[4 * k + 2] = x.z;
            out[4 * k + 3] = x.w;
        }
    } else {
#pragma unroll
        for (int k = 0; k < NF; ++k) out[k] = p[k];
    }
}

// The four slab directions of an octahedron (pairs of opposite faces).
__device__ constexpr double kSlab[4][3] = {{1, 1, 1}, {1, 1, -1}, {1, -1, 1}, {-1, 1, 1}};

// 3x3 inverse (row-major) by the adjugate; returns the determinant.
__device__ inline double inverse3(const double M[9], double N[9]) {
    const double c00 = M[4] * M[8] - M[5] * M[7];
    const double c01 = M[5] * M[6] - M[3] * M[8];
    const double c02 = M[3] * M[7] - M[4] * M[6];
    const double det = M[0] * c00 + M[1] * c01 + M[2] * c02;
    const double id = 1.0 / det;
    N[0] = c00 * id;
    N[1] = (M[2] * M[7] - M[1] * M[8]) * id;
    N[2] = (M[1] * M[5] - M[2] * M[4]) * id;
    N[3] = c01 * id;
    N[4] = (M[0] * M[8] - M[2] * M[6]) * id;
    N[5] = (M[2] * M[3] - M[0] * M[5]) * id;
    N[6] = c02 * id;
    N[7] = (M[1] * M[6] - M[0] * M[7]) * id;
    N[8] = (M[0] * M[4] - M[1] * M[3]) * id;
    return det;
}

// Exact variant: camera-space normals of the primitive's planes, scaled so
// that the octahedron (centre + M s, |s|_1 <= 1, columns of M the offsets
// oc_c) is |n_k . (X - centre)| <= 1 for its 4 slabs, n_k = M^-T kSlab[k],
// and the tetrahedron n_k . (X - centre) <= 1 for the face opposite corner
// k (n_k . oc_m = 1 for the other three corners).  Exact inverses: the
// camera rotation, given in float32, need not be exactly orthonormal.
__device__ inline void exact_normals(int type, const Geom& G, double n[4][3]) {
    if (type == LINPRIM_OCTAHEDRON) {
        double M[9], N[9];
        for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 3; ++c) M[3 * r + c] = G.oc[c][r];
        inverse3(M, N);
#pragma unroll
        for (int k = 0; k < 4; ++k)
#pragma unroll
            for (int r = 0; r < 3; ++r)
                n[k][r] = kSlab[k][0] * N[r] + kSlab[k][1] * N[3 + r] + kSlab[k][2] * N[6 + r];
    } else {
#pragma unroll
        for (int f = 0; f < 4; ++f) {
            double M[9], N[9];
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                const int m = q + (q >= f ? 1 : 0);     // the corners other than f
#pragma unroll
                for (int c = 0; c < 3; ++c) M[3 * q + c] = G.oc[m][c];
            }
            inverse3(M, N);
#pragma unroll
            for (int c = 0; c < 3; ++c) n[f][c] = N[3 * c] + N[3 * c + 1] + N[3 * c + 2];
        }
    }
}

// Smallest |z| component allowed for a face normal relative to its length;
// a face closer to parallel with the viewing rays is treated as this steep.
constexpr double kMinNormalZ = 1e-9;

__device__ inline double clamp_nz(double nz, double nlen) {
    const double lim = kMinNormalZ * nlen;
    if (fabs(nz) >= lim) return nz;
    return nz < 0.0 ? -lim : lim;
}

}  // namespace linprim
