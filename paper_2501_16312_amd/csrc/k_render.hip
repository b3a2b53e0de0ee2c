// k_render.hip -- per-pixel compositing (Sec. 3.2 "Rasterization",
// "Compositing") and its backward pass (Sec. 3.4, App. E).
//
// Work decomposition (gfx950, wave64):
//   * one 64-lane wavefront per screen tile; a TILE x TILE tile is split into
//     (TILE/8)^2 groups of 8 x 8 pixels and lane l owns pixel (l & 7, l >> 3)
//     of every group;
//   * the tile's sorted list is walked in order; the primitive index and the
//     32-dword payload record are wave-uniform and come in through scalar
//     loads (no LDS staging, no barriers);
//   * a group is skipped with scalar compares when the primitive's pixel
//     rectangle misses it, and a pixel is evaluated only inside that
//     rectangle, so images do not depend on the tile size.
//
// Chord.  Pixel rays are parallel to the ray-space z axis, so the ray's
// chord through a convex primitive is max(0, min_up - max_lo): the lowest
// of the planes bounding the primitive from above minus the highest of the
// planes bounding it from below, evaluated at the pixel.  This equals the
// paper's exit-minus-entry Moeller-Trumbore depth difference (the entry and
// exit hits lie on the active lower and upper faces).  Octahedra keep their 8
// faces as 4 slabs (opposite faces are parallel), tetrahedra their 4 faces
// split into upper and lower sets.  Planes are stored relative to the
// primitive's pixel rectangle origin, so ki, kj are small exact integers.
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

__device__ inline int wave_max_int(int v) {
    for (int off = 32; off >= 1; off >>= 1) v = max(v, __shfl_xor(v, off, 64));
    return v;
}

// Round-robin dispatch puts consecutive workgroups on different XCDs; map
// them so that each XCD walks a contiguous run of tiles (neighbouring tiles
// share primitives, and each XCD has its own L2).
__device__ inline int64_t xcd_tile(int64_t b, int64_t nb) {
    constexpr int64_t X = 8;
    const int64_t per = nb / X, rem = nb % X;
    const int64_t x = b % X, loc = b / X;
    return (x < rem) ? x * (per + 1) + loc : rem * (per + 1) + (x - rem) * per + loc;
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

template <int KIND>
__device__ inline void load_rec(const float* __restrict__ rec, Rec& R) {
    R.i0 = __float_as_int(rec[R_I0]);
    R.j0 = __float_as_int(rec[R_J0]);
    R.i1 = __float_as_int(rec[R_I1]);
    R.j1 = __float_as_int(rec[R_J1]);
    R.s2 = rec[R_S2];
    R.r = rec[R_RGB];
    R.g = rec[R_RGB + 1];
    R.b = rec[R_RGB + 2];
    R.fi0 = rec[R_FI0];
    R.fj0 = rec[R_FJ0];
    R.fwi = rec[R_FWI];
    R.fwj = rec[R_FWJ];
    constexpr int NP = (KIND == LINPRIM_OCTAHEDRON) ? 16 : 18;
#pragma unroll
    for (int k = 0; k < NP; ++k) R.p[k] = rec[R_PLANES + k];
    R.sigma = rec[R_SIGMA];
    R.fmap = (KIND == LINPRIM_OCTAHEDRON) ? 0 : __float_as_int(rec[R_FACEMAP]);
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

// Opacity factors of a chord: e = exp(-sigma chord), 1 - o = max(e, 0.01).
__device__ inline float chord_exp(float s2, float delta) {
#pragma clang fp contract(off)
    return __builtin_amdgcn_exp2f(-(s2 * delta));
}

// ---------------------------------------------------------------------------
// Forward.
// ---------------------------------------------------------------------------
template <int TILE, int KIND, bool COUNT>
__global__ __launch_bounds__(64) void k_render_fwd(const ViewInfo* __restrict__ views, int n_views, int64_t n,
                                                   const float* __restrict__ payload, const uint32_t* __restrict__ vals,
                                                   const uint2* __restrict__ ranges, const Status* __restrict__ status,
                                                   uint64_t capacity, float bg0, float bg1, float bg2,
                                                   float* __restrict__ out_rgb, float* __restrict__ out_T,
                                                   int32_t* __restrict__ out_last,
                                                   unsigned long long* __restrict__ counters) {
    if (status->n_pairs > capacity) return;
    constexpr int QX = TILE / 8, NQ = QX * QX;
    const int64_t g = xcd_tile(blockIdx.x, gridDim.x);
    const int v = find_view(views, n_views, g);
    const int W = views[v].width, H = views[v].height, tiles_x = views[v].tiles_x;
    const int64_t lt = g - views[v].tile_base;
    const int tx = (int)(lt % tiles_x), ty = (int)(lt / tiles_x);
    const int lane = threadIdx.x;
    const int lx = lane & 7, ly = lane >> 3;
    const uint2 rg = ranges[g];

    float pxf[NQ], pyf[NQ], T[NQ], C0[NQ], C1[NQ], C2[NQ];
    int last[NQ];
    bool done[NQ];
    uint32_t ev[NQ], hit[NQ], term[NQ];
    uint32_t alive = 0;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        const int x = tx * TILE + (q % QX) * 8 + lx, y = ty * TILE + (q / QX) * 8 + ly;
        const bool valid = x < W && y < H;
        pxf[q] = (float)x;
        pyf[q] = (float)y;
        T[q] = 1.0f;
        C0[q] = C1[q] = C2[q] = 0.0f;
        last[q] = (int)rg.x;
        done[q] = !valid;
        ev[q] = hit[q] = 0;
        term[q] = rg.y;
        if (__ballot(valid)) alive |= 1u << q;
    }
    const float* base = payload + (size_t)v * (size_t)n * kRecordWords;
    for (uint32_t e = rg.x; e < rg.y && alive; ++e) {
        const uint32_t idx = vals[e];
        Rec R;
        load_rec<KIND>(base + (size_t)idx * kRecordWords, R);
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            if (!((alive >> q) & 1u)) continue;
            const int gx0 = tx * TILE + (q % QX) * 8, gy0 = ty * TILE + (q / QX) * 8;
            if (R.i0 > gx0 + 7 || R.i1 < gx0 || R.j0 > gy0 + 7 || R.j1 < gy0) continue;
            if (!done[q]) {
                const float ki = pxf[q] - R.fi0, kj = pyf[q] - R.fj0;
                if (ki >= 0.0f && ki <= R.fwi && kj >= 0.0f && kj <= R.fwj) {
                    if (COUNT) ++ev[q];
                    const float delta = chord_fast<KIND>(R, ki, kj);
                    if (delta > 0.0f) {
                        if (COUNT) ++hit[q];
                        const float ex = chord_exp(R.s2, delta);
                        const float onemo = fmaxf(ex, kOneMinusOMax);
                        const float w = T[q] * (1.0f - onemo);
                        C0[q] = __builtin_fmaf(w, R.r, C0[q]);
                        C1[q] = __builtin_fmaf(w, R.g, C1[q]);
                        C2[q] = __builtin_fmaf(w, R.b, C2[q]);
                        T[q] = T[q] * onemo;
                        last[q] = (int)e + 1;
                        if (T[q] <= kTStop) {
                            done[q] = true;
                            term[q] = e + 1;
                        }
                    }
                }
            }
            if (__ballot(!done[q]) == 0) alive &= ~(1u << q);
        }
    }
    unsigned long long c_it = 0, c_ev = 0, c_hit = 0;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        const int x = tx * TILE + (q % QX) * 8 + lx, y = ty * TILE + (q / QX) * 8 + ly;
        if (x < W && y < H) {
            const int64_t p = (int64_t)y * W + x;
            const int64_t pix = views[v].pix_base + p;
            const int64_t hw = (int64_t)W * H;
            float* o = out_rgb + 3 * views[v].pix_base;
            o[p] = C0[q] + T[q] * bg0;
            o[hw + p] = C1[q] + T[q] * bg1;
            o[2 * hw + p] = C2[q] + T[q] * bg2;
            out_T[pix] = T[q];
            out_last[pix] = last[q];
            if (COUNT) {
                c_it += term[q] - rg.x;
                c_ev += ev[q];
                c_hit += hit[q];
            }
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
// Backward: reverse walk recomputing transmittance, one gradient record of
// kGradWords floats per (tile, primitive) pair.
//   octahedron: [4 s + 0..3] dL/d(A_s, B_s, Dup_s, Dlo_s) for slab s
//   tetrahedron: [3 f + 0..2] dL/d(A_f, B_f, D_f) for face f
//   [16..18] dL/d rgb, [19] dL/d sigma
// ---------------------------------------------------------------------------
__device__ inline int64_t record_slot(const Rec& R, int tile_shift, int tx, int ty, uint32_t prim_offset) {
    const int tx0 = R.i0 >> tile_shift, ty0 = R.j0 >> tile_shift, tx1 = R.i1 >> tile_shift;
    return (int64_t)prim_offset + (int64_t)(ty - ty0) * (tx1 - tx0 + 1) + (tx - tx0);
}

template <int TILE, int KIND>
__global__ __launch_bounds__(64) void k_render_bwd(const ViewInfo* __restrict__ views, int n_views, int64_t n,
                                                   const float* __restrict__ payload, const uint32_t* __restrict__ vals,
                                                   const uint2* __restrict__ ranges, const uint32_t* __restrict__ offsets,
                                                   const Status* __restrict__ status, uint64_t capacity, float bg0,
                                                   float bg1, float bg2, const float* __restrict__ out_T,
                                                   const int32_t* __restrict__ out_last,
                                                   const float* __restrict__ grad_rgb, float* __restrict__ grads) {
    if (status->n_pairs > capacity) return;
    constexpr int QX = TILE / 8, NQ = QX * QX;
    constexpr int SHIFT = (TILE == 8) ? 3 : (TILE == 16) ? 4 : 5;
    const int64_t g = xcd_tile(blockIdx.x, gridDim.x);
    const int v = find_view(views, n_views, g);
    const int W = views[v].width, H = views[v].height, tiles_x = views[v].tiles_x;
    const int64_t lt = g - views[v].tile_base;
    const int tx = (int)(lt % tiles_x), ty = (int)(lt / tiles_x);
    const int lane = threadIdx.x;
    const int lx = lane & 7, ly = lane >> 3;
    const uint2 rg = ranges[g];
    const int64_t hw = (int64_t)W * H;

    float pxf[NQ], pyf[NQ], T[NQ], B0[NQ], B1[NQ], B2[NQ], G0[NQ], G1[NQ], G2[NQ];
    int last[NQ];
    int walk_end = (int)rg.x;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        const int x = tx * TILE + (q % QX) * 8 + lx, y = ty * TILE + (q / QX) * 8 + ly;
        const bool valid = x < W && y < H;
        pxf[q] = (float)x;
        pyf[q] = (float)y;
        T[q] = 1.0f;
        B0[q] = B1[q] = B2[q] = 0.0f;
        G0[q] = G1[q] = G2[q] = 0.0f;
        last[q] = (int)rg.x;
        if (valid) {
            const int64_t p = (int64_t)y * W + x;
            const int64_t pix = views[v].pix_base + p;
            const float* gi = grad_rgb + 3 * views[v].pix_base;
            T[q] = out_T[pix];
            // stay inside this tile's list whatever the caller passed
            last[q] = min(max(out_last[pix], (int)rg.x), (int)rg.y);
            G0[q] = gi[p];
            G1[q] = gi[hw + p];
            G2[q] = gi[2 * hw + p];
            // colour behind the current step (absolute), starts with T_final bg
            B0[q] = T[q] * bg0;
            B1[q] = T[q] * bg1;
            B2[q] = T[q] * bg2;
        }
        walk_end = max(walk_end, last[q]);
    }
    walk_end = wave_max_int(walk_end);
    const float* base = payload + (size_t)v * (size_t)n * kRecordWords;
    const uint32_t* offs = offsets + (size_t)v * (size_t)n;

    // records of entries no pixel of this tile reached are zero
    for (uint32_t e = (uint32_t)walk_end; e < rg.y; ++e) {
        const uint32_t idx = vals[e];
        Rec R;
        load_rec<KIND>(base + (size_t)idx * kRecordWords, R);
        const int64_t slot = record_slot(R, SHIFT, tx, ty, offs[idx]);
        if (lane < kGradWords) grads[slot * kGradWords + lane] = 0.0f;
    }

    for (int e = walk_end - 1; e >= (int)rg.x; --e) {
        const uint32_t idx = vals[e];
        Rec R;
        load_rec<KIND>(base + (size_t)idx * kRecordWords, R);
        float acc[kGradWords];
#pragma unroll
        for (int k = 0; k < kGradWords; ++k) acc[k] = 0.0f;
        bool contributed = false;
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            const int gx0 = tx * TILE + (q % QX) * 8, gy0 = ty * TILE + (q / QX) * 8;
            if (R.i0 > gx0 + 7 || R.i1 < gx0 || R.j0 > gy0 + 7 || R.j1 < gy0) continue;
            if (e >= last[q]) continue;
            const float ki = pxf[q] - R.fi0, kj = pyf[q] - R.fj0;
            if (!(ki >= 0.0f && ki <= R.fwi && kj >= 0.0f && kj <= R.fwj)) continue;
            int ih, il;
            const float delta = chord<KIND>(R, ki, kj, ih, il);
            if (!(delta > 0.0f)) continue;
            const float ex = chord_exp(R.s2, delta);
            const float onemo = fmaxf(ex, kOneMinusOMax);
            const float o = 1.0f - onemo;
            const float ro = __builtin_amdgcn_rcpf(onemo);
            const float Tk = T[q] * ro;                 // transmittance in front of this primitive
            // dC/do = T_k rgb - behind / (1 - o)
            const float dLdo = G0[q] * (Tk * R.r - B0[q] * ro) + G1[q] * (Tk * R.g - B1[q] * ro) +
                               G2[q] * (Tk * R.b - B2[q] * ro);
            const float wk = Tk * o;
            acc[16] += G0[q] * wk;
            acc[17] += G1[q] * wk;
            acc[18] += G2[q] * wk;
            B0[q] += wk * R.r;
            B1[q] += wk * R.g;
            B2[q] += wk * R.b;
            T[q] = Tk;
            contributed = true;
            if (ex >= kOneMinusOMax) {                   // not clamped: o = 1 - exp(-sigma chord)
                const float gD = dLdo * R.sigma * ex;    // dL/dchord
                acc[19] += dLdo * delta * ex;            // dL/dsigma
                if (KIND == LINPRIM_OCTAHEDRON) {
#pragma unroll
                    for (int s = 0; s < 4; ++s) {
                        const float gh = (ih == s) ? gD : 0.0f;
                        const float gl = (il == s) ? gD : 0.0f;
                        const float d = gh - gl;
                        acc[4 * s + 0] += d * ki;
                        acc[4 * s + 1] += d * kj;
                        acc[4 * s + 2] += gh;
                        acc[4 * s + 3] -= gl;
                    }
                } else {
                    const int fh = (R.fmap >> (2 * ih)) & 3;
                    const int fl = (R.fmap >> (2 * (il + 3))) & 3;
#pragma unroll
                    for (int f = 0; f < 4; ++f) {
                        const float d = ((fh == f) ? gD : 0.0f) - ((fl == f) ? gD : 0.0f);
                        acc[3 * f + 0] += d * ki;
                        acc[3 * f + 1] += d * kj;
                        acc[3 * f + 2] += d;
                    }
                }
            }
        }
        const int64_t slot = record_slot(R, SHIFT, tx, ty, offs[idx]);
        float outv = 0.0f;
        if (__ballot(contributed) != 0) {
#pragma unroll
            for (int k = 0; k < kGradWords; ++k) {
                const float tot = wave_sum(acc[k]);
                outv = (lane == k) ? tot : outv;
            }
        }
        if (lane < kGradWords) grads[slot * kGradWords + lane] = outv;
    }
}

// ---------------------------------------------------------------------------
// Launchers.
// ---------------------------------------------------------------------------
template <int TILE, int KIND>
static void fwd_dispatch(bool count, dim3 grid, hipStream_t s, const ViewInfo* views, int nv, int64_t n,
                         const float* payload, const uint32_t* vals, const uint2* ranges, const Status* st,
                         uint64_t cap, const float bg[3], float* rgb, float* T, int32_t* last,
                         unsigned long long* counters) {
    if (count)
        hipLaunchKernelGGL((k_render_fwd<TILE, KIND, true>), grid, dim3(64), 0, s, views, nv, n, payload, vals, ranges,
                           st, cap, bg[0], bg[1], bg[2], rgb, T, last, counters);
    else
        hipLaunchKernelGGL((k_render_fwd<TILE, KIND, false>), grid, dim3(64), 0, s, views, nv, n, payload, vals, ranges,
                           st, cap, bg[0], bg[1], bg[2], rgb, T, last, counters);
}

hipError_t launch_render_fwd_ex(const ViewLayout& L, const char* vws, const PairLayout& P, const char* pws,
                                int result_in_b, int type, int tile, int32_t n_views, const float bg[3],
                                float* out_rgb, float* out_T, int32_t* out_last, unsigned long long* counters,
                                hipStream_t stream) {
    if (L.n_tiles_total == 0) return hipSuccess;
    const ViewInfo* views = reinterpret_cast<const ViewInfo*>(vws + L.views);
    const float* payload = reinterpret_cast<const float*>(vws + L.payload);
    const uint32_t* vals = reinterpret_cast<const uint32_t*>(pws + (result_in_b ? P.vals_b : P.vals_a));
    const uint2* ranges = reinterpret_cast<const uint2*>(vws + L.ranges);
    const Status* st = reinterpret_cast<const Status*>(vws + L.status);
    const uint64_t cap = (uint64_t)P.capacity;
    dim3 grid((unsigned)L.n_tiles_total);
    const bool count = counters != nullptr;
    if (type == LINPRIM_OCTAHEDRON) {
        if (tile == 8) fwd_dispatch<8, 0>(count, grid, stream, views, n_views, L.n, payload, vals, ranges, st, cap, bg, out_rgb, out_T, out_last, counters);
        else if (tile == 16) fwd_dispatch<16, 0>(count, grid, stream, views, n_views, L.n, payload, vals, ranges, st, cap, bg, out_rgb, out_T, out_last, counters);
        else fwd_dispatch<32, 0>(count, grid, stream, views, n_views, L.n, payload, vals, ranges, st, cap, bg, out_rgb, out_T, out_last, counters);
    } else {
        if (tile == 8) fwd_dispatch<8, 1>(count, grid, stream, views, n_views, L.n, payload, vals, ranges, st, cap, bg, out_rgb, out_T, out_last, counters);
        else if (tile == 16) fwd_dispatch<16, 1>(count, grid, stream, views, n_views, L.n, payload, vals, ranges, st, cap, bg, out_rgb, out_T, out_last, counters);
        else fwd_dispatch<32, 1>(count, grid, stream, views, n_views, L.n, payload, vals, ranges, st, cap, bg, out_rgb, out_T, out_last, counters);
    }
    return hipGetLastError();
}

hipError_t launch_render_fwd(const ViewLayout& L, const char* vws, const PairLayout& P, const char* pws,
                             int result_in_b, int type, int tile, int32_t n_views, const float bg[3],
                             float* out_rgb, float* out_T, int32_t* out_last, hipStream_t stream) {
    return launch_render_fwd_ex(L, vws, P, pws, result_in_b, type, tile, n_views, bg, out_rgb, out_T, out_last,
                                nullptr, stream);
}

template <int TILE, int KIND>
static void bwd_dispatch(dim3 grid, hipStream_t s, const ViewInfo* views, int nv, int64_t n, const float* payload,
                         const uint32_t* vals, const uint2* ranges, const uint32_t* offsets, const Status* st,
                         uint64_t cap, const float bg[3], const float* T, const int32_t* last, const float* grad,
                         float* grads) {
    hipLaunchKernelGGL((k_render_bwd<TILE, KIND>), grid, dim3(64), 0, s, views, nv, n, payload, vals, ranges, offsets,
                       st, cap, bg[0], bg[1], bg[2], T, last, grad, grads);
}

hipError_t launch_render_bwd(const ViewLayout& L, const char* vws, const PairLayout& P, char* pws, int result_in_b,
                             int type, int tile, int32_t n_views, const float bg[3], const float* out_T,
                             const int32_t* out_last, const float* grad_rgb, hipStream_t stream) {
    if (L.n_tiles_total == 0) return hipSuccess;
    const ViewInfo* views = reinterpret_cast<const ViewInfo*>(vws + L.views);
    const float* payload = reinterpret_cast<const float*>(vws + L.payload);
    const uint32_t* vals = reinterpret_cast<const uint32_t*>(pws + (result_in_b ? P.vals_b : P.vals_a));
    const uint2* ranges = reinterpret_cast<const uint2*>(vws + L.ranges);
    const uint32_t* offsets = reinterpret_cast<const uint32_t*>(vws + L.offsets);
    const Status* st = reinterpret_cast<const Status*>(vws + L.status);
    float* grads = reinterpret_cast<float*>(pws + P.grads);
    const uint64_t cap = (uint64_t)P.capacity;
    dim3 grid((unsigned)L.n_tiles_total);
    if (type == LINPRIM_OCTAHEDRON) {
        if (tile == 8) bwd_dispatch<8, 0>(grid, stream, views, n_views, L.n, payload, vals, ranges, offsets, st, cap, bg, out_T, out_last, grad_rgb, grads);
        else if (tile == 16) bwd_dispatch<16, 0>(grid, stream, views, n_views, L.n, payload, vals, ranges, offsets, st, cap, bg, out_T, out_last, grad_rgb, grads);
        else bwd_dispatch<32, 0>(grid, stream, views, n_views, L.n, payload, vals, ranges, offsets, st, cap, bg, out_T, out_last, grad_rgb, grads);
    } else {
        if (tile == 8) bwd_dispatch<8, 1>(grid, stream, views, n_views, L.n, payload, vals, ranges, offsets, st, cap, bg, out_T, out_last, grad_rgb, grads);
        else if (tile == 16) bwd_dispatch<16, 1>(grid, stream, views, n_views, L.n, payload, vals, ranges, offsets, st, cap, bg, out_T, out_last, grad_rgb, grads);
        else bwd_dispatch<32, 1>(grid, stream, views, n_views, L.n, payload, vals, ranges, offsets, st, cap, bg, out_T, out_last, grad_rgb, grads);
    }
    return hipGetLastError();
}

}  // namespace linprim
