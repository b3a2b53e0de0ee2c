// k_render.hip -- per-pixel compositing (Sec. 3.2 "Rasterization",
// "Compositing") and its backward pass (Sec. 3.4, App. E).
//
// Work decomposition (gfx950, wave64):
//   * one 64-lane wavefront per 8 x 8 pixel group; a TILE x TILE screen tile
//     has (TILE/8)^2 groups, each an independent workgroup; lane l owns pixel
//     (l & 7, l >> 3) of its group;
//   * the tile's sorted list is walked in batches of 64 entries: one vector
//     load brings 64 primitive indices (and, for tiles wider than a group,
//     their pixel rectangles), a ballot keeps the entries whose rectangle
//     meets the group, and only those entries' 32-dword payloads are read,
//     wave-uniform, through scalar loads issued one entry ahead (no LDS, no
//     barriers);
//   * a pixel is evaluated only inside the primitive's pixel rectangle, so
//     images do not depend on the tile size.
//
// Chord.  Pixel rays are parallel to the ray-space z axis, so the ray's
// chord through a convex primitive is max(0, min_up - max_lo): the lowest
// of the planes bounding the primitive from above minus the highest of the
// planes bounding it from below, evaluated at the pixel.  This equals the
// paper's exit-minus-entry Moeller-Trumbore depth difference (the entry and
// exit hits lie on the active lower and upper faces).  Octahedra keep their 8
// faces as 4 slabs (opposite faces are parallel), tetrahedra their 4 faces
// split into upper and lower sets.  Planes are stored relative to the
// centre of the primitive's pixel rectangle, so ki, kj are small exact
// half-integers.
#include "linprim_common.h"

namespace linprim {

// ---------------------------------------------------------------------------
// Wave helpers.
// ---------------------------------------------------------------------------
template <int CTRL, int ROW_MASK = 0xF>
__device__ inline float dpp_move(float src) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(src), CTRL, ROW_MASK, 0xF, false));
}

// Sum over the 64 lanes; every lane must be active.  Returns the total (uniform).
__device__ inline float wave_sum(float v) {
    v += dpp_move<0xB1>(v);          // quad_perm(1,0,3,2)
    v += dpp_move<0x4E>(v);          // quad_perm(2,3,0,1)
    v += dpp_move<0x141>(v);         // row_half_mirror
    v += dpp_move<0x140>(v);         // row_mirror: every lane holds its row sum
    v += dpp_move<0x142, 0xA>(v);    // row_bcast:15 -> rows 1 and 3
    v += dpp_move<0x143, 0x8>(v);    // row_bcast:31 -> row 3 holds the total
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}

// s_waitcnt lgkmcnt(0) (vmcnt and expcnt left at their maxima), fenced so
// that the scheduler moves no scalar load above it.
__device__ inline void smem_wait_all() {
    __builtin_amdgcn_sched_barrier(0);
    __builtin_amdgcn_s_waitcnt(0xC07F);
    __builtin_amdgcn_sched_barrier(0);
}
__device__ inline void sched_fence() { __builtin_amdgcn_sched_barrier(0); }

__device__ inline int wave_max_int(int v) {
    for (int off = 32; off >= 1; off >>= 1) v = max(v, __shfl_xor(v, off, 64));
    return v;
}

// Round-robin dispatch puts consecutive workgroups on different XCDs.  Deal
// out chunks of kXcdChunk consecutive waves (neighbouring tiles, which share
// primitives) round-robin instead, so each XCD's L2 sees whole chunks while
// every XCD still gets a spread of the image (tiles differ a lot in work).
constexpr int64_t kXcdChunk = 32;
__device__ inline int64_t xcd_tile(int64_t b, int64_t nb) {
    constexpr int64_t X = 8;
    const int64_t full = (nb / (X * kXcdChunk)) * (X * kXcdChunk);
    if (b >= full) return b;
    const int64_t x = b % X, k = b / X;
    return ((k / kXcdChunk) * X + x) * kXcdChunk + (k % kXcdChunk);
}

__device__ inline int find_view(const ViewInfo* __restrict__ views, int n_views, int64_t g) {
    int lo = 0, hi = n_views - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (views[mid].tile_base <= g) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// ---------------------------------------------------------------------------
// Chords.  Contraction is disabled inside so the forward and the backward
// kernels evaluate bit-identical chords; fused multiply-adds are explicit.
// ---------------------------------------------------------------------------
struct Rec {
    int i0, j0, i1, j1;
    float s2, r, g, b, fi0, fj0, fwi, fwj;
    float p[18];
    float sigma;
    int fmap;
};

template <int KIND, bool EXACT = false, bool RECT = true>
__device__ inline void load_rec(const float* __restrict__ rec, Rec& R) {
    if (RECT) {
        R.i0 = __float_as_int(rec[R_I0]);
        R.j0 = __float_as_int(rec[R_J0]);
        R.i1 = __float_as_int(rec[R_I1]);
        R.j1 = __float_as_int(rec[R_J1]);
    } else {
        R.i0 = R.j0 = R.i1 = R.j1 = 0;
    }
    R.s2 = rec[R_S2];
    R.r = rec[R_RGB];
    R.g = rec[R_RGB + 1];
    R.b = rec[R_RGB + 2];
    R.fi0 = rec[R_FI0];
    R.fj0 = rec[R_FJ0];
    R.fwi = rec[R_FWI];
    R.fwj = rec[R_FWJ];
    constexpr int NP = (EXACT || KIND == LINPRIM_OCTAHEDRON) ? 16 : 18;
#pragma unroll
    for (int k = 0; k < NP; ++k) R.p[k] = rec[R_PLANES + k];
    R.sigma = rec[R_SIGMA];
    R.fmap = (EXACT || KIND == LINPRIM_OCTAHEDRON) ? 0 : __float_as_int(rec[R_FACEMAP]);
}

// Returns hi - lo; ih / il are the active upper / lower slot (first on ties).
template <int KIND>
__device__ inline float chord(const Rec& R, float ki, float kj, int& ih, int& il) {
#pragma clang fp contract(off)
    if (KIND == LINPRIM_OCTAHEDRON) {
        float hi = 0.f, lo = 0.f;
        ih = 0; il = 0;
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const float u = __builtin_fmaf(R.p[4 * s + 0], ki, R.p[4 * s + 1] * kj);
            const float h = u + R.p[4 * s + 2];
            const float l = u + R.p[4 * s + 3];
            if (s == 0) { hi = h; lo = l; }
            else {
                if (h < hi) { hi = h; ih = s; }
                if (l > lo) { lo = l; il = s; }
            }
        }
        return hi - lo;
    } else {
        float hi = 0.f, lo = 0.f;
        ih = 0; il = 0;
#pragma unroll
        for (int s = 0; s < 3; ++s) {
            const float h = __builtin_fmaf(R.p[3 * s + 0], ki, __builtin_fmaf(R.p[3 * s + 1], kj, R.p[3 * s + 2]));
            const float l = __builtin_fmaf(R.p[9 + 3 * s + 0], ki, __builtin_fmaf(R.p[9 + 3 * s + 1], kj, R.p[9 + 3 * s + 2]));
            if (s == 0) { hi = h; lo = l; }
            else {
                if (h < hi) { hi = h; ih = s; }
                if (l > lo) { lo = l; il = s; }
            }
        }
        return hi - lo;
    }
}

// Same chord without slot tracking (forward).
template <int KIND>
__device__ inline float chord_fast(const Rec& R, float ki, float kj) {
#pragma clang fp contract(off)
    if (KIND == LINPRIM_OCTAHEDRON) {
        float h[4], l[4];
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const float u = __builtin_fmaf(R.p[4 * s + 0], ki, R.p[4 * s + 1] * kj);
            h[s] = u + R.p[4 * s + 2];
            l[s] = u + R.p[4 * s + 3];
        }
        const float hi = fminf(fminf(h[0], h[1]), fminf(h[2], h[3]));
        const float lo = fmaxf(fmaxf(l[0], l[1]), fmaxf(l[2], l[3]));
        return hi - lo;
    } else {
        float h[3], l[3];
#pragma unroll
        for (int s = 0; s < 3; ++s) {
            h[s] = __builtin_fmaf(R.p[3 * s + 0], ki, __builtin_fmaf(R.p[3 * s + 1], kj, R.p[3 * s + 2]));
            l[s] = __builtin_fmaf(R.p[9 + 3 * s + 0], ki, __builtin_fmaf(R.p[9 + 3 * s + 1], kj, R.p[9 + 3 * s + 2]));
        }
        return fminf(fminf(h[0], h[1]), h[2]) - fmaxf(fmaxf(l[0], l[1]), l[2]);
    }
}

// Same chord, also returning the entry depth lo (relative to the centre's
// ray-space depth) for the depth map.
template <int KIND>
__device__ inline float chord_entry(const Rec& R, float ki, float kj, float& lo_out) {
#pragma clang fp contract(off)
    if (KIND == LINPRIM_OCTAHEDRON) {
        float h[4], l[4];
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const float u = __builtin_fmaf(R.p[4 * s + 0], ki, R.p[4 * s + 1] * kj);
            h[s] = u + R.p[4 * s + 2];
            l[s] = u + R.p[4 * s + 3];
        }
        const float hi = fminf(fminf(h[0], h[1]), fminf(h[2], h[3]));
        const float lo = fmaxf(fmaxf(l[0], l[1]), fmaxf(l[2], l[3]));
        lo_out = lo;
        return hi - lo;
    } else {
        float h[3], l[3];
#pragma unroll
        for (int s = 0; s < 3; ++s) {
            h[s] = __builtin_fmaf(R.p[3 * s + 0], ki, __builtin_fmaf(R.p[3 * s + 1], kj, R.p[3 * s + 2]));
            l[s] = __builtin_fmaf(R.p[9 + 3 * s + 0], ki, __builtin_fmaf(R.p[9 + 3 * s + 1], kj, R.p[9 + 3 * s + 2]));
        }
        const float lo = fmaxf(fmaxf(l[0], l[1]), l[2]);
        lo_out = lo;
        return fminf(fminf(h[0], h[1]), h[2]) - lo;
    }
}

// Exact variant (no ray space): each plane k bounds the relative depth tau
// along the pixel ray at (u_k + h) / (c_k - u_k).  Per plane: u, 1/(c - u),
// the plane's upper and lower bounds (a tetrahedron face is an exit where
// c - u >= 0, an entry elsewhere; the other bound is infinite).  A plane
// parallel to the ray gives infinite (or, on its boundary, NaN) bounds,
// which the min / max reductions ignore.
struct ExactPlanes {
    float u[4], inv[4], hi[4], lo[4];
    float U, L;
};

template <int KIND>
__device__ inline void exact_planes(const Rec& R, float ki, float kj, ExactPlanes& X) {
#pragma clang fp contract(off)
    X.U = INFINITY;
    X.L = -INFINITY;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const float u = __builtin_fmaf(R.p[4 * k + 0], ki, __builtin_fmaf(R.p[4 * k + 1], kj, R.p[4 * k + 2]));
        const float den = R.p[4 * k + 3] - u;
        const float inv = __builtin_amdgcn_rcpf(den);
        X.u[k] = u;
        X.inv[k] = inv;
        if (KIND == LINPRIM_OCTAHEDRON) {
            const float ui = u * inv;
            const float t1 = ui - inv, t2 = ui + inv;
            X.hi[k] = fmaxf(t1, t2);
            X.lo[k] = fminf(t1, t2);
        } else {
            const float t = __builtin_fmaf(u, inv, inv);
            const bool ex = den >= 0.0f;
            X.hi[k] = ex ? t : INFINITY;
            X.lo[k] = ex ? -INFINITY : t;
        }
        X.U = fminf(X.U, X.hi[k]);
        X.L = fmaxf(X.L, X.lo[k]);
    }
}

// |D| (min exits - max entries) with rn = |D| of the pixel ray; the z_c
// factor of the chord is folded into the record's sigma.
__device__ inline float exact_chord(const ExactPlanes& X, float rn) {
#pragma clang fp contract(off)
    return (X.U - X.L) * rn;
}

// Opacity factors of a chord: e = exp(-sigma chord), 1 - o = max(e, 0.01).
__device__ inline float chord_exp(float s2, float delta) {
#pragma clang fp contract(off)
    return __builtin_amdgcn_exp2f(-(s2 * delta));
}

// |D| of the exact variant's pixel ray D = ((x + 1/2 - cx)/fx, (y + 1/2 - cy)/fy, 1).
__device__ inline float ray_norm(const ViewInfo& V, int x, int y) {
    const float rx = (float)(((double)x + 0.5 - V.cx) / V.fx);
    const float ry = (float)(((double)y + 0.5 - V.cy) / V.fy);
    return sqrtf(rx * rx + ry * ry + 1.0f);
}

// ---------------------------------------------------------------------------
// Wave placement: wave w (XCD-chunked) handles group q = w % NQ of the tile at
// position w / NQ of a render order.  The forward's: heavy tiles first, then
// the others, each part in tile order, so that consecutive positions are
// mostly neighbouring tiles.  The backward's (also taken by the exact
// variant's forward): longest lists first in classes of list length (tile
// order inside a class), so that the waves that start last are short and
// the kernel has no long tail.
// ---------------------------------------------------------------------------
struct Place {
    int v, tx, ty, gx0, gy0, W, H, q;
    int64_t g;
};

template <int TILE>
__device__ inline Place place_wave(const ViewInfo* __restrict__ views, int n_views, const uint32_t* __restrict__ order) {
    constexpr int QX = TILE / 8, NQ = QX * QX;
    const int64_t w = xcd_tile(blockIdx.x, gridDim.x);
    Place P;
    P.g = order[w / NQ];
    P.q = (int)(w % NQ);
    P.v = find_view(views, n_views, P.g);
    P.W = views[P.v].width;
    P.H = views[P.v].height;
    const int tiles_x = views[P.v].tiles_x;
    const int64_t lt = P.g - views[P.v].tile_base;
    P.tx = (int)(lt % tiles_x);
    P.ty = (int)(lt / tiles_x);
    P.gx0 = P.tx * TILE + (P.q % QX) * 8;
    P.gy0 = P.ty * TILE + (P.q / QX) * 8;
    return P;
}

__device__ inline bool rect_meets_group(int4 r, int gx0, int gy0) {
    return !(r.x > gx0 + 7 || r.z < gx0 || r.y > gy0 + 7 || r.w < gy0);
}

// One batch of up to 64 list entries starting at e0: lane l holds entry
// e0 + l's primitive index (and, for the backward, the index of the
// gradient record of that (tile, primitive) pair and this group).
struct Batch {
    uint32_t idx;
    uint32_t off;      // gradient record index (backward only)
    uint64_t mask;     // entries whose pixel rectangle meets the group
    uint32_t touch;    // words of the entries' records read only to bring them into L2
};

// Gradient records of a slot are laid out by tile of its tile rectangle
// (row-major), NQ groups per tile, from the slot's pair offset on.
__device__ inline uint32_t record_index(int4 r, int tile_shift, int tx, int ty, uint32_t prim_offset, int NQ, int q) {
    const int tx0 = r.x >> tile_shift, ty0 = r.y >> tile_shift, tx1 = r.z >> tile_shift;
    return (prim_offset + (uint32_t)((ty - ty0) * (tx1 - tx0 + 1) + (tx - tx0))) * (uint32_t)NQ + (uint32_t)q;
}

template <int NQ, bool WANT_OFF>
__device__ inline Batch load_batch(const float* __restrict__ base, const uint32_t* __restrict__ vals,
                                   const uint32_t* __restrict__ offs, uint32_t e0, uint32_t nb, int gx0, int gy0,
                                   int tile_shift = 0, int tx = 0, int ty = 0, int q = 0) {
    const int lane = threadIdx.x;
    Batch B;
    B.idx = 0;
    B.off = 0;
    B.touch = 0;
    bool rel = false;
    if ((uint32_t)lane < nb) {
        B.idx = vals[e0 + lane];
        const float* rp = base + (size_t)B.idx * kRecordWords;
        if (NQ == 1 && !WANT_OFF) {
            rel = true;   // every entry of a group-sized tile meets it
            B.touch = __float_as_uint(rp[0]);
        } else {
            const int4 r = *reinterpret_cast<const int4*>(rp);
            rel = (NQ == 1) || rect_meets_group(r, gx0, gy0);
            if (WANT_OFF) B.off = record_index(r, tile_shift, tx, ty, offs[B.idx], NQ, q);
        }
        // the record's second 64-byte line, for the scalar loads that follow
        if (rel) B.touch ^= __float_as_uint(rp[16]);
    }
    B.mask = __ballot(rel);
    return B;
}

// ---------------------------------------------------------------------------
// Forward.
// ---------------------------------------------------------------------------
// Depth maps of the appendix "Depth and Surface Reconstruction": the
// distance along the pixel ray to the entry of the first primitive at which
// the cumulative opacity exceeds 0.5.  The walk keeps that primitive's entry
// depth relative to its centre (ray space: the highest lower plane, whose
// depth axis is the distance from the camera; exact rays: the entry
// parameter tau); the centre's depth is added once per pixel afterwards.
constexpr float kDepthT = 0.5f;

__device__ inline double centre_depth(const ViewInfo& V, const float* __restrict__ means, uint32_t prim, bool exact) {
    const double x = means[3 * (size_t)prim], y = means[3 * (size_t)prim + 1], z = means[3 * (size_t)prim + 2];
    const double t0 = V.Rw[0] * x + V.Rw[1] * y + V.Rw[2] * z + V.tw[0];
    const double t1 = V.Rw[3] * x + V.Rw[4] * y + V.Rw[5] * z + V.tw[1];
    const double t2 = V.Rw[6] * x + V.Rw[7] * y + V.Rw[8] * z + V.tw[2];
    return exact ? t2 : sqrt(t0 * t0 + t1 * t1 + t2 * t2);
}

template <int TILE, int KIND, bool COUNT, bool EXACT, bool DEPTH>
__global__ __launch_bounds__(64) void k_render_fwd(const ViewInfo* __restrict__ views, int n_views, int64_t n,
                                                   const float* __restrict__ payload, const uint32_t* __restrict__ vals,
                                                   const uint2* __restrict__ ranges, const Status* __restrict__ status,
                                                   uint64_t capacity, float bg0, float bg1, float bg2,
                                                   float* __restrict__ out_rgb, float* __restrict__ out_T,
                                                   int32_t* __restrict__ out_last,
                                                   unsigned long long* __restrict__ counters,
                                                   const float* __restrict__ means,
                                                   float* __restrict__ out_depth, const uint32_t* __restrict__ order) {
    if (status->n_pairs > capacity) return;
    constexpr int QX = TILE / 8, NQ = QX * QX;
    const Place P = place_wave<TILE>(views, n_views, order);
    if (P.gx0 >= P.W || P.gy0 >= P.H) return;
    const int lane = threadIdx.x;
    const int x = P.gx0 + (lane & 7), y = P.gy0 + (lane >> 3);
    const bool valid = x < P.W && y < P.H;
    const float pxf = (float)x, pyf = (float)y;
    const float rn = EXACT ? ray_norm(views[P.v], x, y) : 1.0f;
    const uint2 rg = ranges[P.g];
    float T = 1.0f, C0 = 0.0f, C1 = 0.0f, C2 = 0.0f;
    int last = (int)rg.x;
    // lanes still compositing, as a wave-uniform mask (kept in scalar
    // registers; each lane's bit is read back with an inverse ballot)
    uint64_t live = __builtin_amdgcn_ballot_w64(valid);
    uint32_t ev = 0, hit = 0, term = rg.y;
    uint32_t half = 0xffffffffu;   // list position at which 1 - T first exceeds 0.5
    float half_entry = 0.0f;       // its entry depth relative to its centre
    const float* base = payload + (size_t)P.v * (size_t)n * kRecordWords;
    bool alive = true;
    uint32_t sink = 0;   // keeps the L2-warming loads alive; never stored
    Batch nxt = load_batch<NQ, false>(base, vals, nullptr, rg.x, min(64u, rg.y - rg.x), P.gx0, P.gy0);
    for (uint32_t e0 = rg.x; e0 < rg.y && alive; e0 += 64) {
        Batch cur = nxt;
        const uint32_t e1 = e0 + 64;
        if (e1 < rg.y) nxt = load_batch<NQ, false>(base, vals, nullptr, e1, min(64u, rg.y - e1), P.gx0, P.gy0);
        sink ^= cur.touch;
        uint64_t mask = cur.mask;
        if (!mask) continue;
        // Two record buffers used in turn: the next surviving entry's record
        // is loaded into one while the other is blended, with no copies.
        auto blend = [&](const Rec& R, uint32_t e) {
            // Branch-free: lanes that do not see the primitive blend with
            // 1 - o = 1 exactly, which leaves C and T unchanged.
            const float ki = pxf - R.fi0, kj = pyf - R.fj0;
            // bitwise &: every test is a plain compare, no short-circuit branches
            // lane masks of single compares combine in scalar registers
            const uint64_t m_in = __builtin_amdgcn_ballot_w64(fabsf(ki) <= R.fwi) &
                                  __builtin_amdgcn_ballot_w64(fabsf(kj) <= R.fwj) & live;
            const bool inside = __builtin_amdgcn_inverse_ballot_w64(m_in);
            float dch, entry = 0.0f;
            if (EXACT) {
                ExactPlanes X;
                exact_planes<KIND>(R, ki, kj, X);
                dch = exact_chord(X, rn);
                entry = X.L;
            } else if (DEPTH) {
                dch = chord_entry<KIND>(R, ki, kj, entry);
            } else {
                dch = chord_fast<KIND>(R, ki, kj);
            }
            const uint64_t m_hit = m_in & __builtin_amdgcn_ballot_w64(dch > 0.0f);
            const bool hitp = __builtin_amdgcn_inverse_ballot_w64(m_hit);
            if (COUNT) {
                ev += inside ? 1u : 0u;
                hit += hitp ? 1u : 0u;
            }
            const float ex = hitp ? chord_exp(R.s2, dch) : 1.0f;
            const float onemo = fmaxf(ex, kOneMinusOMax);
            const float w = T * (1.0f - onemo);
            C0 = __builtin_fmaf(w, R.r, C0);
            C1 = __builtin_fmaf(w, R.g, C1);
            C2 = __builtin_fmaf(w, R.b, C2);
            if (DEPTH) {
                const bool cross = T >= kDepthT && T * onemo < kDepthT;
                half = cross ? e : half;
                half_entry = cross ? entry : half_entry;
            }
            T = T * onemo;
            last = hitp ? (int)e + 1 : last;
            // T only falls where the primitive was hit
            const uint64_t stop = __builtin_amdgcn_ballot_w64(T <= kTStop) & m_hit;
            if (COUNT) term = __builtin_amdgcn_inverse_ballot_w64(stop) ? e + 1 : term;
            live &= ~stop;
            return live != 0;
        };
        auto next_rec = [&](Rec& R) {
            const int b = __builtin_ctzll(mask);
            mask &= mask - 1;
            load_rec<KIND, EXACT>(base + (size_t)(uint32_t)__builtin_amdgcn_readlane((int)cur.idx, b) * kRecordWords, R);
            return e0 + (uint32_t)b;
        };
        // Scalar loads complete out of order, so waiting for one buffer means
        // waiting for every scalar load in flight: wait first, then issue
        // the next record's load, then blend from the buffer just waited for.
        Rec RA, RB;
        uint32_t eA = next_rec(RA), eB = 0;
        while (true) {
            smem_wait_all();
            const bool haveB = mask != 0;
            if (haveB) eB = next_rec(RB);
            sched_fence();
            if (!blend(RA, eA)) { alive = false; break; }
            if (!haveB) break;
            smem_wait_all();
            const bool haveA = mask != 0;
            if (haveA) eA = next_rec(RA);
            sched_fence();
            if (!blend(RB, eB)) { alive = false; break; }
            if (!haveA) break;
        }
    }
    if (n < 0) out_T[0] = __uint_as_float(sink);   // n >= 0: never taken
    unsigned long long c_it = 0, c_ev = 0, c_hit = 0;
    if (valid) {
        const int64_t p = (int64_t)y * P.W + x;
        const int64_t pix = views[P.v].pix_base + p;
        const int64_t hw = (int64_t)P.W * P.H;
        float* o = out_rgb + 3 * views[P.v].pix_base;
        o[p] = C0 + T * bg0;
        o[hw + p] = C1 + T * bg1;
        o[2 * hw + p] = C2 + T * bg2;
        out_T[pix] = T;
        out_last[pix] = last;
        if (DEPTH) {
            float dz = 0.0f;
            if (half != 0xffffffffu) {
                const double zc = centre_depth(views[P.v], means, vals[half], EXACT);
                // exact rays: camera depth z_c (1 + tau) times |D|
                dz = EXACT ? (float)((zc + zc * (double)half_entry) * (double)rn) : (float)(zc + (double)half_entry);
            }
            out_depth[pix] = dz;
        }
        if (COUNT) {
            c_it = term - rg.x;
            c_ev = ev;
            c_hit = hit;
        }
    }
    if (COUNT) {
        const float fi = wave_sum((float)c_it), fe = wave_sum((float)c_ev), fh = wave_sum((float)c_hit);
        if (lane == 0) {
            atomicAdd(counters + 0, (unsigned long long)fi);
            atomicAdd(counters + 1, (unsigned long long)fe);
            atomicAdd(counters + 2, (unsigned long long)fh);
        }
    }
}

// ---------------------------------------------------------------------------
// Backward: reverse walk recomputing transmittance.  One gradient record of
// kGradWords floats per (tile, primitive) pair and group, at
// (pair slot) * NQ + q, written for every entry whose rectangle meets the
// group (zeros if no pixel of the group reached it):
//   octahedron: [4 s + 0..3] dL/d(A_s, B_s, Dup_s, Dlo_s) for slab s
//   tetrahedron: [3 f + 0..2] dL/d(A_f, B_f, D_f) for face f
//   [16..18] dL/d rgb, [19] dL/d sigma
// ---------------------------------------------------------------------------

// One step of the backward walk for this lane's pixel, branch-free: a lane
// that does not see the primitive (not active, outside the rectangle, zero
// chord) runs the same instructions with delta = 0, o = 0, 1 - o = 1, which
// leaves T and the colour behind (GB = dL/dC . colour behind) unchanged
// exactly and yields zero terms.  Writes the lane's gradient terms of the
// entry's record into acc; returns whether the lane contributed.
template <int KIND, bool EXACT>
__device__ inline bool bwd_step(const Rec& R, bool active, float pxf, float pyf, float rn, float G0, float G1,
                                float G2, float& T, float& GB, float (&acc)[kGradWords]) {
    const float ki = pxf - R.fi0, kj = pyf - R.fj0;
    const bool inside = active & (fabsf(ki) <= R.fwi) & (fabsf(kj) <= R.fwj);
    // chord and the active (lowest upper, highest lower) planes,
    // the first one in plane order on ties; the chord is the same
    // number the forward computed
    float dch;
    bool eh[4], el[4];
    int ih = 0, il = 0;
    ExactPlanes X;
    if (EXACT) {
        exact_planes<KIND>(R, ki, kj, X);
        dch = exact_chord(X, rn);
        bool fh = false, fl = false;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            eh[k] = !fh && X.hi[k] == X.U;
            el[k] = !fl && X.lo[k] == X.L;
            fh = fh || eh[k];
            fl = fl || el[k];
        }
    } else if (KIND == LINPRIM_OCTAHEDRON) {
#pragma clang fp contract(off)
        float h[4], l[4];
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const float u = __builtin_fmaf(R.p[4 * s + 0], ki, R.p[4 * s + 1] * kj);
            h[s] = u + R.p[4 * s + 2];
            l[s] = u + R.p[4 * s + 3];
        }
        const float hi = fminf(fminf(h[0], h[1]), fminf(h[2], h[3]));
        const float lo = fmaxf(fmaxf(l[0], l[1]), fmaxf(l[2], l[3]));
        dch = hi - lo;
        bool fh = false, fl = false;
#pragma unroll
        for (int s = 0; s < 3; ++s) {
            eh[s] = !fh && h[s] == hi;
            el[s] = !fl && l[s] == lo;
            fh = fh || eh[s];
            fl = fl || el[s];
        }
        eh[3] = !fh;
        el[3] = !fl;
    } else {
        dch = chord<KIND>(R, ki, kj, ih, il);
    }
    const bool contributed = inside && dch > 0.0f;
    const float delta = contributed ? dch : 0.0f;
    const float ex = contributed ? chord_exp(R.s2, delta) : 1.0f;
    const float onemo = fmaxf(ex, kOneMinusOMax);
    const float o = 1.0f - onemo;
    const float ro = __builtin_amdgcn_rcpf(onemo);
    const float Tk = T * ro;                     // transmittance in front of this primitive
    // dL/do = G . (T_k rgb - behind / (1 - o))
    const float Grgb = G0 * R.r + G1 * R.g + G2 * R.b;
    const float dLdo = Tk * Grgb - ro * GB;
    const float wk = Tk * o;
    acc[16] = G0 * wk;
    acc[17] = G1 * wk;
    acc[18] = G2 * wk;
    GB += wk * Grgb;
    T = Tk;
    // not clamped: o = 1 - exp(-sigma chord)
    const bool open = contributed && ex >= kOneMinusOMax;
    const float q = dLdo * ex;
    const float gD = open ? q * R.sigma : 0.0f;    // dL/dchord
    acc[19] = open ? q * delta : 0.0f;             // dL/dsigma
    if (EXACT) {
        // words 4 k + 0..3: dL/d(a_k, b_k, g_k, c_k); a plane bound
        // tau = (u + h) / (c - u) has dtau/du = (c + h) / (c - u)^2
        // and dtau/dc = -tau / (c - u)
        const float g = gD * rn;                   // dL/d(U - L)
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const float c = R.p[4 * k + 3];
            const float inv = X.inv[k];
            const float ge = eh[k] ? g : 0.0f, gl = el[k] ? g : 0.0f;
            float gu;
            if (KIND == LINPRIM_OCTAHEDRON) {
                // the upper bound has h = +1 where c - u >= 0, else h = -1
                const float hh = (c - X.u[k] >= 0.0f) ? 1.0f : -1.0f;
                gu = (ge * (c + hh) - gl * (c - hh)) * (inv * inv);
            } else {
                gu = (ge - gl) * (c + 1.0f) * (inv * inv);
            }
            const float gc = (gl * X.L - ge * X.U) * inv;
            const bool act = eh[k] || el[k];
            const float Gu = act ? gu : 0.0f, Gc = act ? gc : 0.0f;
            acc[4 * k + 0] = Gu * ki;
            acc[4 * k + 1] = Gu * kj;
            acc[4 * k + 2] = Gu;
            acc[4 * k + 3] = Gc;
        }
    } else if (KIND == LINPRIM_OCTAHEDRON) {
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const float gh = eh[s] ? gD : 0.0f;
            const float gl = el[s] ? gD : 0.0f;
            const float d = gh - gl;
            acc[4 * s + 0] = d * ki;
            acc[4 * s + 1] = d * kj;
            acc[4 * s + 2] = gh;
            acc[4 * s + 3] = gl;                   // negated after the reduction
        }
    } else {
        const int fh = (R.fmap >> (2 * ih)) & 3;
        const int fl = (R.fmap >> (2 * (il + 3))) & 3;
#pragma unroll
        for (int f = 0; f < 4; ++f) {
            const float d = ((fh == f) ? gD : 0.0f) - ((fl == f) ? gD : 0.0f);
            acc[3 * f + 0] = d * ki;
            acc[3 * f + 1] = d * kj;
            acc[3 * f + 2] = d;
        }
#pragma unroll
        for (int k = 12; k < 16; ++k) acc[k] = 0.0f;
    }
    return contributed;
}

template <int TILE, int KIND, bool EXACT>
__global__ __launch_bounds__(64) void k_render_bwd(const ViewInfo* __restrict__ views, int n_views, int64_t n,
                                                   const float* __restrict__ payload, const uint32_t* __restrict__ vals,
                                                   const uint2* __restrict__ ranges, const uint32_t* __restrict__ offsets,
                                                   const Status* __restrict__ status, uint64_t capacity, float bg0,
                                                   float bg1, float bg2, const float* __restrict__ out_T,
                                                   const int32_t* __restrict__ out_last,
                                                   const float* __restrict__ grad_rgb, float* __restrict__ grads,
                                                   const uint32_t* __restrict__ order) {
    if (status->n_pairs > capacity) return;
    constexpr int QX = TILE / 8, NQ = QX * QX;
    constexpr int SHIFT = (TILE == 8) ? 3 : (TILE == 16) ? 4 : 5;
    const Place P = place_wave<TILE>(views, n_views, order);
    if (P.gx0 >= P.W || P.gy0 >= P.H) return;
    const int lane = threadIdx.x;
    const int x = P.gx0 + (lane & 7), y = P.gy0 + (lane >> 3);
    const bool valid = x < P.W && y < P.H;
    const float pxf = (float)x, pyf = (float)y;
    const float rn = EXACT ? ray_norm(views[P.v], x, y) : 1.0f;
    const uint2 rg = ranges[P.g];
    const int64_t hw = (int64_t)P.W * P.H;
    const float* base = payload + (size_t)P.v * (size_t)n * kRecordWords;
    const uint32_t* offs = offsets + (size_t)P.v * (size_t)n;

    // GB = dL/dC . (colour behind the current step), kept as one running
    // dot product (the colour behind itself is not needed)
    float T = 1.0f, GB = 0.0f, G0 = 0.0f, G1 = 0.0f, G2 = 0.0f;
    int last = (int)rg.x;
    if (valid) {
        const int64_t p = (int64_t)y * P.W + x;
        const int64_t pix = views[P.v].pix_base + p;
        const float* gi = grad_rgb + 3 * views[P.v].pix_base;
        T = out_T[pix];
        // stay inside this tile's list whatever the caller passed
        last = min(max(out_last[pix], (int)rg.x), (int)rg.y);
        G0 = gi[p];
        G1 = gi[hw + p];
        G2 = gi[2 * hw + p];
        // the colour behind starts as T_final bg
        GB = T * (G0 * bg0 + G1 * bg1 + G2 * bg2);
    }
    const uint32_t walk_end = (uint32_t)wave_max_int(last);

    // zero records of the entries that meet the group but no pixel reached
    for (uint32_t e0 = walk_end; e0 < rg.y; e0 += 64) {
        const Batch bt = load_batch<NQ, true>(base, vals, offs, e0, min(64u, rg.y - e0), P.gx0, P.gy0, SHIFT, P.tx,
                                              P.ty, P.q);
        uint64_t mask = bt.mask;
        while (mask) {
            const int b = __builtin_ctzll(mask);
            mask &= mask - 1;
            const uint32_t slot = (uint32_t)__builtin_amdgcn_readlane((int)bt.off, b);
            if (lane < kGradWords) grads[(size_t)slot * kGradWords + lane] = 0.0f;
        }
    }

    for (uint32_t e_hi = walk_end; e_hi > rg.x;) {
        const uint32_t nb = min(64u, e_hi - rg.x);
        const uint32_t e0 = e_hi - nb;
        e_hi = e0;
        const Batch bt = load_batch<NQ, true>(base, vals, offs, e0, nb, P.gx0, P.gy0, SHIFT, P.tx, P.ty, P.q);
        uint64_t mask = bt.mask;
        if (!mask) continue;
        // Entries in reverse order, two record buffers used in turn (see the
        // forward for the wait / load order).
        auto next_rec = [&](Rec& R) {
            const int b = 63 - __builtin_clzll(mask);
            mask &= ~(1ull << b);
            load_rec<KIND, EXACT, false>(base + (size_t)(uint32_t)__builtin_amdgcn_readlane((int)bt.idx, b) *
                                             kRecordWords, R);
            return b;
        };
        auto step = [&](const Rec& R, int bcur) {
            const uint32_t e = e0 + (uint32_t)bcur;
            // a lane past its last blended entry takes no part
            float acc[kGradWords];
            const bool contributed = bwd_step<KIND, EXACT>(R, (int)e < last, pxf, pyf, rn, G0, G1, G2, T, GB, acc);
            const size_t slot = (uint32_t)__builtin_amdgcn_readlane((int)bt.off, bcur);
            float outv = 0.0f;
            if (__ballot(contributed) != 0) outv = wave_reduce20(acc, lane);
            const int ridx = reduce20_index(lane);
            // octahedra: words 4 s + 3 are dL/dDlo = -sum of the lower-plane terms
            if (!EXACT && KIND == LINPRIM_OCTAHEDRON && ridx < 16 && (ridx & 3) == 3) outv = -outv;
            if (ridx >= 0) grads[slot * kGradWords + ridx] = outv;
        };
        Rec RA, RB;
        int bA = next_rec(RA), bB = 0;
        while (true) {
            smem_wait_all();
            const bool haveB = mask != 0;
            if (haveB) bB = next_rec(RB);
            sched_fence();
            step(RA, bA);
            if (!haveB) break;
            smem_wait_all();
            const bool haveA = mask != 0;
            if (haveA) bA = next_rec(RA);
            sched_fence();
            step(RB, bB);
            if (!haveA) break;
        }
    }
}

// ---------------------------------------------------------------------------
// Backward of the exact variant: each 16-lane row of the wave owns one 4 x 4
// quad of the 8 x 8 group and walks, in reverse list order, only the entries
// whose rectangle meets its quad and that lie before the last blended entry
// of one of its pixels; the four rows walk independently, so a step
// evaluates up to four entries.  The list is taken in batches of kBwdBatch
// entries: the batch's records (words 4..31) are staged in LDS, a row reads
// the record of its current entry from there, sums its 16 lanes' gradient
// terms (transposed, inside the row) and adds them to the entry's LDS
// accumulator, the rows one after the other (a fixed order); the batch's
// records are then written out, one per lane.  Same records as
// k_render_bwd.  The exact step is heavy enough that skipping the entries a
// quad does not meet pays for the LDS round trips; the ray-space step is not.
// ---------------------------------------------------------------------------
constexpr int kBwdBatch = 32;
static_assert(kBwdBatch <= 32, "entry masks are 32-bit");

// Sums 20 values over the 16 lanes of each row, transposed: four DPP steps
// each halve the values a lane keeps (row mirror: lane i with 15 - i, split
// on bit 3; half-row mirror: i with 7 - i, bit 2; quad swaps i with i ^ 2,
// bit 1, and i with i ^ 1, bit 0).  With base = 10 b3 + 5 b2 of the row lane
// index, a lane ends with the totals of words
//   b1 b0 = 00: base, base + 1;  01: base + 2;  10: base + 3, base + 4;
//   11: none.
__device__ inline void row_reduce20(const float (&v)[20], int li, float& t0, float& t1, int& w0, int& w1) {
    const bool h3 = (li >> 3) & 1, h2 = (li >> 2) & 1, h1 = (li >> 1) & 1, h0 = li & 1;
    float a[10];
#pragma unroll
    for (int j = 0; j < 10; ++j) {
        const float keep = h3 ? v[j + 10] : v[j];
        const float give = h3 ? v[j] : v[j + 10];
        a[j] = keep + dpp_move<0x140>(give);
    }
    float b[6];
#pragma unroll
    for (int j = 0; j < 5; ++j) {
        const float keep = h2 ? a[j + 5] : a[j];
        const float give = h2 ? a[j] : a[j + 5];
        b[j] = keep + dpp_move<0x141>(give);
    }
    b[5] = 0.0f;
    float c[4];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        const float keep = h1 ? b[j + 3] : b[j];
        const float give = h1 ? b[j] : b[j + 3];
        c[j] = keep + dpp_move<0x4E>(give);
    }
    c[3] = 0.0f;
    float d[2];
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        const float keep = h0 ? c[j + 2] : c[j];
        const float give = h0 ? c[j] : c[j + 2];
        d[j] = keep + dpp_move<0xB1>(give);
    }
    const int base = 10 * (int)h3 + 5 * (int)h2;
    t0 = d[0];
    t1 = d[1];
    if (!h1 && !h0) { w0 = base; w1 = base + 1; }
    else if (!h1) { w0 = base + 2; w1 = -1; }
    else if (!h0) { w0 = base + 3; w1 = base + 4; }
    else { w0 = -1; w1 = -1; }
}

template <int TILE, int KIND, bool EXACT>
__global__ __launch_bounds__(64) void k_render_bwd_rows(const ViewInfo* __restrict__ views, int n_views, int64_t n,
                                                   const float* __restrict__ payload, const uint32_t* __restrict__ vals,
                                                   const uint2* __restrict__ ranges, const uint32_t* __restrict__ offsets,
                                                   const Status* __restrict__ status, uint64_t capacity, float bg0,
                                                   float bg1, float bg2, const float* __restrict__ out_T,
                                                   const int32_t* __restrict__ out_last,
                                                   const float* __restrict__ grad_rgb, float* __restrict__ grads,
                                                   const uint32_t* __restrict__ order) {
    __shared__ float4 srec[kBwdBatch][7];             // record words 4..31
    __shared__ float sacc[kBwdBatch][kGradWords];     // gradient record accumulators
    if (status->n_pairs > capacity) return;
    constexpr int QX = TILE / 8, NQ = QX * QX;
    constexpr int SHIFT = (TILE == 8) ? 3 : (TILE == 16) ? 4 : 5;
    const Place P = place_wave<TILE>(views, n_views, order);
    if (P.gx0 >= P.W || P.gy0 >= P.H) return;
    const int lane = threadIdx.x, row = lane >> 4, li = lane & 15;
    // row r owns the quad (r & 1, r >> 1) of the group
    const int x = P.gx0 + 4 * (row & 1) + (li & 3), y = P.gy0 + 4 * (row >> 1) + (li >> 2);
    const bool valid = x < P.W && y < P.H;
    const float pxf = (float)x, pyf = (float)y;
    const float rn = EXACT ? ray_norm(views[P.v], x, y) : 1.0f;
    const uint2 rg = ranges[P.g];
    const int64_t hw = (int64_t)P.W * P.H;
    const float* base = payload + (size_t)P.v * (size_t)n * kRecordWords;
    const uint32_t* offs = offsets + (size_t)P.v * (size_t)n;

    // GB = dL/dC . (colour behind the current step), kept as one running
    // dot product (the colour behind itself is not needed)
    float T = 1.0f, GB = 0.0f, G0 = 0.0f, G1 = 0.0f, G2 = 0.0f;
    int last = (int)rg.x;
    if (valid) {
        const int64_t p = (int64_t)y * P.W + x;
        const int64_t pix = views[P.v].pix_base + p;
        const float* gi = grad_rgb + 3 * views[P.v].pix_base;
        T = out_T[pix];
        // stay inside this tile's list whatever the caller passed
        last = min(max(out_last[pix], (int)rg.x), (int)rg.y);
        G0 = gi[p];
        G1 = gi[hw + p];
        G2 = gi[2 * hw + p];
        // the colour behind starts as T_final bg
        GB = T * (G0 * bg0 + G1 * bg1 + G2 * bg2);
    }
    const uint32_t walk_end = (uint32_t)wave_max_int(last);
    // each row's end: the largest last blended position of its 16 pixels
    int rlast = last;
#pragma unroll
    for (int m = 8; m >= 1; m >>= 1) rlast = max(rlast, __shfl_xor(rlast, m, 16));
    const uint32_t rend[4] = {(uint32_t)__builtin_amdgcn_readlane(rlast, 0),
                              (uint32_t)__builtin_amdgcn_readlane(rlast, 16),
                              (uint32_t)__builtin_amdgcn_readlane(rlast, 32),
                              (uint32_t)__builtin_amdgcn_readlane(rlast, 48)};

    // zero records of the entries that meet the group but no pixel reached
    for (uint32_t e0 = walk_end; e0 < rg.y; e0 += 64) {
        const Batch bt = load_batch<NQ, true>(base, vals, offs, e0, min(64u, rg.y - e0), P.gx0, P.gy0, SHIFT, P.tx,
                                              P.ty, P.q);
        uint64_t mask = bt.mask;
        while (mask) {
            const int b = __builtin_ctzll(mask);
            mask &= mask - 1;
            const uint32_t slot = (uint32_t)__builtin_amdgcn_readlane((int)bt.off, b);
            if (lane < kGradWords) grads[(size_t)slot * kGradWords + lane] = 0.0f;
        }
    }

    for (uint32_t e_hi = walk_end; e_hi > rg.x;) {
        const uint32_t nb = min((uint32_t)kBwdBatch, e_hi - rg.x);
        const uint32_t e0 = e_hi - nb;
        e_hi = e0;
        // lane l < nb stages entry e0 + l: its record, a zero accumulator, and
        // the quads whose row walks it
        bool meets = false;
        uint32_t qm = 0, off = 0;
        if ((uint32_t)lane < nb) {
            const uint32_t idx = vals[e0 + lane];
            const float* rp = base + (size_t)idx * kRecordWords;
            const int4 r = *reinterpret_cast<const int4*>(rp);
            meets = (NQ == 1) || rect_meets_group(r, P.gx0, P.gy0);
            if (meets) {
                off = record_index(r, SHIFT, P.tx, P.ty, offs[idx], NQ, P.q);
                const float4* src = reinterpret_cast<const float4*>(rp + 4);
#pragma unroll
                for (int k = 0; k < 7; ++k) srec[lane][k] = src[k];
                float4* acc4 = reinterpret_cast<float4*>(sacc[lane]);
#pragma unroll
                for (int k = 0; k < kGradWords / 4; ++k) acc4[k] = make_float4(0.f, 0.f, 0.f, 0.f);
                const uint32_t e = e0 + (uint32_t)lane;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int qx0 = P.gx0 + 4 * (q & 1), qy0 = P.gy0 + 4 * (q >> 1);
                    const bool mq = !(r.x > qx0 + 3 || r.z < qx0 || r.y > qy0 + 3 || r.w < qy0);
                    qm |= (mq && e < rend[q]) ? (1u << q) : 0u;
                }
            }
        }
        const uint32_t staged = (uint32_t)__ballot(meets);   // kBwdBatch <= 32 entries
        if (staged == 0) continue;
        // a staged entry: the record a row without an entry reads (finite
        // values, so that its lanes' state stays exactly unchanged)
        const int bsafe = __builtin_ctz(staged);
        const uint32_t m0 = (uint32_t)__ballot(qm & 1u), m1 = (uint32_t)__ballot(qm & 2u),
                       m2 = (uint32_t)__ballot(qm & 4u), m3 = (uint32_t)__ballot(qm & 8u);
        uint32_t mask = (row == 0) ? m0 : (row == 1) ? m1 : (row == 2) ? m2 : m3;
        while (true) {
            const bool act = mask != 0;
            if (__ballot(act) == 0) break;
            // the row's next entry, in reverse order (a row without one runs
            // the step with every lane outside)
            const int bcur = act ? 31 - __builtin_clz(mask) : bsafe;
            mask &= act ? ~(1u << bcur) : ~0u;
            Rec R;
            {
                const float4 w0 = srec[bcur][0], w1 = srec[bcur][1];
                R.s2 = w0.x; R.r = w0.y; R.g = w0.z; R.b = w0.w;
                R.fi0 = w1.x; R.fj0 = w1.y; R.fwi = w1.z; R.fwj = w1.w;
                float pw[20];
#pragma unroll
                for (int k = 0; k < 5; ++k) {
                    const float4 w = srec[bcur][2 + k];
                    pw[4 * k] = w.x; pw[4 * k + 1] = w.y; pw[4 * k + 2] = w.z; pw[4 * k + 3] = w.w;
                }
#pragma unroll
                for (int k = 0; k < 18; ++k) R.p[k] = pw[k];
                R.sigma = pw[R_SIGMA - R_PLANES];
                R.fmap = (EXACT || KIND == LINPRIM_OCTAHEDRON) ? 0 : __float_as_int(pw[R_FACEMAP - R_PLANES]);
                R.i0 = R.j0 = R.i1 = R.j1 = 0;
            }
            const uint32_t e = e0 + (uint32_t)bcur;
            float acc[kGradWords];
            const bool contributed = bwd_step<KIND, EXACT>(R, act && (int)e < last, pxf, pyf, rn, G0, G1, G2, T, GB, acc);
            if (__ballot(contributed) != 0) {
                float t0, t1;
                int w0, w1;
                row_reduce20(acc, li, t0, t1, w0, w1);
                // the rows one after the other: a fixed order of the additions
#pragma unroll
                for (int rr = 0; rr < 4; ++rr) {
                    if (row == rr && act) {
                        if (w0 >= 0) atomicAdd(&sacc[bcur][w0], t0);
                        if (w1 >= 0) atomicAdd(&sacc[bcur][w1], t1);
                    }
                }
            }
        }
        // the batch's records, one per lane (octahedra: words 4 s + 3 are
        // dL/dDlo = -sum of the lower-plane terms)
        if (meets) {
            const float4* acc4 = reinterpret_cast<const float4*>(sacc[lane]);
            float4* dst = reinterpret_cast<float4*>(grads + (size_t)off * kGradWords);
#pragma unroll
            for (int k = 0; k < kGradWords / 4; ++k) {
                float4 o = acc4[k];
                if (!EXACT && KIND == LINPRIM_OCTAHEDRON && k < 4) o.w = -o.w;
                dst[k] = o;
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Launchers.
// ---------------------------------------------------------------------------
template <int TILE>
static dim3 wave_grid(const ViewLayout& L) {
    constexpr int NQ = (TILE / 8) * (TILE / 8);
    return dim3((unsigned)(L.n_tiles_total * NQ));
}

template <int TILE, int KIND, bool EXACT>
static void fwd_dispatch(bool count, const ViewLayout& Lv, hipStream_t s, const ViewInfo* views, int nv, int64_t n,
                         const float* payload, const uint32_t* vals, const uint2* ranges, const Status* st,
                         uint64_t cap, const float bg[3], float* rgb, float* T, int32_t* last,
                         unsigned long long* counters, const float* means, float* depth, const uint32_t* order) {
    const dim3 grid = wave_grid<TILE>(Lv);
#define LP_K(C_, D_)                                                                                              \
    hipLaunchKernelGGL((k_render_fwd<TILE, KIND, C_, EXACT, D_>), grid, dim3(64), 0, s, views, nv, n, payload, vals, \
                       ranges, st, cap, bg[0], bg[1], bg[2], rgb, T, last, counters, means, depth, order)
    if (depth) {
        if (count) LP_K(true, true); else LP_K(false, true);
    } else {
        if (count) LP_K(true, false); else LP_K(false, false);
    }
#undef LP_K
}

hipError_t launch_render_fwd_ex(const ViewLayout& L, const char* vws, const PairLayout& P, const char* pws,
                                int result_in_b, int type, bool exact, int tile, int32_t n_views, const float bg[3],
                                float* out_rgb, float* out_T, int32_t* out_last, float* out_depth,
                                const float* means, unsigned long long* counters, hipStream_t stream) {
    if (L.n_tiles_total == 0) return hipSuccess;
    const ViewInfo* views = reinterpret_cast<const ViewInfo*>(vws + L.views);
    const float* payload = reinterpret_cast<const float*>(vws + L.payload);
    const uint32_t* vals = reinterpret_cast<const uint32_t*>(pws + (result_in_b ? P.vals_b : P.vals_a));
    const uint2* ranges = reinterpret_cast<const uint2*>(vws + L.ranges);
    const Status* st = reinterpret_cast<const Status*>(vws + L.status);
    // the exact variant's heavier step runs best in the backward's order
    const uint32_t* order = reinterpret_cast<const uint32_t*>(vws + (exact ? L.order_bwd : L.order));
    const uint64_t cap = (uint64_t)P.capacity;
    const bool count = counters != nullptr;
#define LP_FWD(T_, K_, E_) fwd_dispatch<T_, K_, E_>(count, L, stream, views, n_views, L.n, payload, vals, ranges, st, \
                                                    cap, bg, out_rgb, out_T, out_last, counters, means, out_depth, order)
#define LP_FWD_T(K_, E_)                                                       \
    do {                                                                       \
        if (tile == 8) LP_FWD(8, K_, E_);                                      \
        else if (tile == 16) LP_FWD(16, K_, E_);                               \
        else LP_FWD(32, K_, E_);                                               \
    } while (0)
    if (type == LINPRIM_OCTAHEDRON) {
        if (exact) LP_FWD_T(0, true); else LP_FWD_T(0, false);
    } else {
        if (exact) LP_FWD_T(1, true); else LP_FWD_T(1, false);
    }
#undef LP_FWD_T
#undef LP_FWD
    return hipGetLastError();
}

hipError_t launch_render_fwd(const ViewLayout& L, const char* vws, const PairLayout& P, const char* pws,
                             int result_in_b, int type, bool exact, int tile, int32_t n_views, const float bg[3],
                             float* out_rgb, float* out_T, int32_t* out_last, hipStream_t stream) {
    return launch_render_fwd_ex(L, vws, P, pws, result_in_b, type, exact, tile, n_views, bg, out_rgb, out_T, out_last,
                                nullptr, nullptr, nullptr, stream);
}

template <int TILE, int KIND, bool EXACT>
static void bwd_dispatch(const ViewLayout& Lv, hipStream_t s, const ViewInfo* views, int nv, int64_t n,
                         const float* payload, const uint32_t* vals, const uint2* ranges, const uint32_t* offsets,
                         const Status* st, uint64_t cap, const float bg[3], const float* T, const int32_t* last,
                         const float* grad, float* grads, const uint32_t* order) {
    if (EXACT)
        hipLaunchKernelGGL((k_render_bwd_rows<TILE, KIND, true>), wave_grid<TILE>(Lv), dim3(64), 0, s, views, nv, n,
                           payload, vals, ranges, offsets, st, cap, bg[0], bg[1], bg[2], T, last, grad, grads, order);
    else
        hipLaunchKernelGGL((k_render_bwd<TILE, KIND, false>), wave_grid<TILE>(Lv), dim3(64), 0, s, views, nv, n,
                           payload, vals, ranges, offsets, st, cap, bg[0], bg[1], bg[2], T, last, grad, grads, order);
}

hipError_t launch_render_bwd(const ViewLayout& L, const char* vws, const PairLayout& P, char* pws, int result_in_b,
                             int type, bool exact, int tile, int32_t n_views, const float bg[3], const float* out_T,
                             const int32_t* out_last, const float* grad_rgb, hipStream_t stream) {
    if (L.n_tiles_total == 0) return hipSuccess;
    const ViewInfo* views = reinterpret_cast<const ViewInfo*>(vws + L.views);
    const float* payload = reinterpret_cast<const float*>(vws + L.payload);
    const uint32_t* vals = reinterpret_cast<const uint32_t*>(pws + (result_in_b ? P.vals_b : P.vals_a));
    const uint2* ranges = reinterpret_cast<const uint2*>(vws + L.ranges);
    const uint32_t* offsets = reinterpret_cast<const uint32_t*>(vws + L.offsets);
    const Status* st = reinterpret_cast<const Status*>(vws + L.status);
    float* grads = reinterpret_cast<float*>(pws + P.grads);
    const uint32_t* order = reinterpret_cast<const uint32_t*>(vws + L.order_bwd);
    const uint64_t cap = (uint64_t)P.capacity;
#define LP_BWD(T_, K_, E_) bwd_dispatch<T_, K_, E_>(L, stream, views, n_views, L.n, payload, vals, ranges, offsets, \
                                                    st, cap, bg, out_T, out_last, grad_rgb, grads, order)
#define LP_BWD_T(K_, E_)                                                       \
    do {                                                                       \
        if (tile == 8) LP_BWD(8, K_, E_);                                      \
        else if (tile == 16) LP_BWD(16, K_, E_);                               \
        else LP_BWD(32, K_, E_);                                               \
    } while (0)
    if (type == LINPRIM_OCTAHEDRON) {
        if (exact) LP_BWD_T(0, true); else LP_BWD_T(0, false);
    } else {
        if (exact) LP_BWD_T(1, true); else LP_BWD_T(1, false);
    }
#undef LP_BWD_T
#undef LP_BWD
    return hipGetLastError();
}

}  // namespace linprim
