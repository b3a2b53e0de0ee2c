// k_preprocess.hip -- per-primitive preprocessing (Sec. 3.2 "Preprocessing")
// and the prefix sum of the per-primitive tile counts.
//
// Compiled with -ffp-contract=off: the pixel rectangles and depth keys are
// integer decisions taken in IEEE double precision with the fixed
// expression order of build_geometry().
#include "linprim_common.h"

namespace linprim {

// Per-view constants of up to kViewChunk views, computed on the host in
// double precision and passed by value.
void fill_view_chunk(const linprim_camera* cams, int v0, int cnt, int tile, int64_t& tile_base, int64_t& pix_base,
                     ViewChunk& ch) {
    for (int k = 0; k < cnt; ++k) {
        const linprim_camera& c = cams[v0 + k];
        ViewInfo& V = ch.v[k];
        for (int r = 0; r < 3; ++r) {
            for (int q = 0; q < 3; ++q) V.Rw[3 * r + q] = (double)c.world_to_cam[4 * r + q];
            V.tw[r] = (double)c.world_to_cam[4 * r + 3];
        }
        // camera position -R^T t
        for (int q = 0; q < 3; ++q)
            V.cam_pos[q] = -(V.Rw[q] * V.tw[0] + V.Rw[3 + q] * V.tw[1] + V.Rw[6 + q] * V.tw[2]);
        V.fx = c.fx; V.fy = c.fy; V.cx = c.cx; V.cy = c.cy;
        V.near_z = c.near_z;
        V.width = c.width; V.height = c.height;
        V.tiles_x = (c.width + tile - 1) / tile;
        V.tiles_y = (c.height + tile - 1) / tile;
        V.tile_base = tile_base;
        V.pix_base = pix_base;
        tile_base += (int64_t)V.tiles_x * V.tiles_y;
        pix_base += (int64_t)c.width * c.height;
    }
}

__global__ void k_store_views(ViewChunk chunk, int count, ViewInfo* __restrict__ dst) {
    const int i = threadIdx.x;
    if (i < count) dst[i] = chunk.v[i];
}

hipError_t launch_store_views(const linprim_camera* cams, int32_t n_views, int tile, ViewInfo* views,
                              hipStream_t stream) {
    int64_t tile_base = 0, pix_base = 0;
    for (int v0 = 0; v0 < n_views; v0 += kViewChunk) {
        ViewChunk ch;
        const int cnt = (n_views - v0) < kViewChunk ? (n_views - v0) : kViewChunk;
        fill_view_chunk(cams, v0, cnt, tile, tile_base, pix_base, ch);
        hipLaunchKernelGGL(k_store_views, dim3(1), dim3(64), 0, stream, ch, cnt, views + v0);
    }
    return hipGetLastError();
}

// The geometric part of k_preprocess for slot `slot` (view V): the record
// except its colour, the depth key and the tile count.  Returns whether the
// primitive is visible in the view.
template <int KIND, bool EXACT>
__device__ inline bool preprocess_view(bool ok, Geom& G, const float* mu, double sigma, const ViewInfo& V,
                                       int64_t slot, int tile_shift, int aa, float* __restrict__ payload,
                                       uint32_t* __restrict__ depth_keys, uint32_t* __restrict__ tiles,
                                       uint2* __restrict__ trect) {
    float* rec = payload + slot * kRecordWords;
    if (!ok || !build_view(KIND, EXACT, aa != 0, mu, V, G)) {
        // culled: no tiles; the record is left as it was (nothing reads it)
        depth_keys[slot] = 0u;
        tiles[slot] = 0u;
        return false;
    }
    const int i0 = G.rect[0], j0 = G.rect[1], i1 = G.rect[2], j1 = G.rect[3];
    const uint32_t ntile = (uint32_t)((i1 >> tile_shift) - (i0 >> tile_shift) + 1) *
                           (uint32_t)((j1 >> tile_shift) - (j0 >> tile_shift) + 1);
    depth_keys[slot] = G.key;
    tiles[slot] = ntile;
    trect[slot] = pack_tile_rect(i0, j0, i1, j1, tile_shift);

    float out[kRecordWords];
    for (int k = 0; k < kRecordWords; ++k) out[k] = 0.0f;
    out[R_I0] = __int_as_float(i0);
    out[R_J0] = __int_as_float(j0);
    out[R_I1] = __int_as_float(i1);
    out[R_J1] = __int_as_float(j1);
    out[R_S2] = (float)(sigma * kLog2e);
    out[R_FI0] = 0.5f * (float)(i0 + i1);
    out[R_FJ0] = 0.5f * (float)(j0 + j1);
    out[R_FWI] = 0.5f * (float)(i1 - i0);
    out[R_FWJ] = 0.5f * (float)(j1 - j0);
    out[R_SIGMA] = (float)sigma;

    // Offsets of the rectangle centre's pixel position from the ray-space
    // centre: the render kernels evaluate planes at the half-integers
    // ki = i - (i0 + i1)/2, kj = j - (j0 + j1)/2, so that the float32
    // offsets, and the plane values they multiply, stay within half the
    // rectangle.
    const double ox = 0.5 * (double)(i0 + i1) + 0.5 - G.c[0];
    const double oy = 0.5 * (double)(j0 + j1) + 0.5 - G.c[1];
    if (EXACT) {
        // camera-space planes along the pixel ray X = z_c (1 + tau) D: with
        // the projected centre (G.c[0], G.c[1]) and dx = i + 1/2 - c_x,
        // n . (centre - z_c D) = -z_c (n_x dx / fx + n_y dy / fy)
        double nrm[4][3];
        exact_normals(KIND, G, nrm);
        const double zc = G.tc[2];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const double a = -zc * nrm[k][0] / V.fx, b = -zc * nrm[k][1] / V.fy;
            out[R_PLANES + 4 * k + 0] = (float)a;
            out[R_PLANES + 4 * k + 1] = (float)b;
            out[R_PLANES + 4 * k + 2] = (float)(a * ox + b * oy);
            out[R_PLANES + 4 * k + 3] = (float)(nrm[k][0] * G.tc[0] + nrm[k][1] * G.tc[1] + nrm[k][2] * G.tc[2]);
        }
        out[R_S2] = (float)(sigma * zc * kLog2e);
        out[R_SIGMA] = (float)(sigma * zc);
    } else if (KIND == LINPRIM_OCTAHEDRON) {
        // primitive = c + M s, |s|_1 <= 1, M = [a0 a1 a2]; the pair of faces
        // with sign pattern sg is the slab |sg . M^-1 (X - c)| <= 1.
        double M[9], N[9];
        for (int r = 0; r < 3; ++r)
            for (int k = 0; k < 3; ++k) M[3 * r + k] = G.a[k][r];
        inverse3(M, N);
        for (int s = 0; s < 4; ++s) {
            double nu[3];
            for (int c = 0; c < 3; ++c)
                nu[c] = kSlab[s][0] * N[c] + kSlab[s][1] * N[3 + c] + kSlab[s][2] * N[6 + c];
            const double nl = sqrt(nu[0] * nu[0] + nu[1] * nu[1] + nu[2] * nu[2]);
            const double nz = clamp_nz(nu[2], nl);
            const double inz = 1.0 / nz;
            const double A = -nu[0] * inz, B = -nu[1] * inz, W = fabs(inz);
            const double ctr = A * ox + B * oy;
            out[R_PLANES + 4 * s + 0] = (float)A;
            out[R_PLANES + 4 * s + 1] = (float)B;
            out[R_PLANES + 4 * s + 2] = (float)(ctr + W);
            out[R_PLANES + 4 * s + 3] = (float)(ctr - W);
        }
    } else {
        // face f holds the three corners other than f; its outward normal
        // decides whether it bounds the ray from above (n_z > 0) or below.
        double pA[4], pB[4], pD[4];
        int up[4], lo[4], nu = 0, nl = 0;
        for (int f = 0; f < 4; ++f) {
            int m[3], q = 0;
            for (int k = 0; k < 4; ++k)
                if (k != f) m[q++] = k;
            const double* P0 = G.a[m[0]];
            const double e1[3] = {G.a[m[1]][0] - P0[0], G.a[m[1]][1] - P0[1], G.a[m[1]][2] - P0[2]};
            const double e2[3] = {G.a[m[2]][0] - P0[0], G.a[m[2]][1] - P0[1], G.a[m[2]][2] - P0[2]};
            double nv[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2], e1[0] * e2[1] - e1[1] * e2[0]};
            const double to_f = nv[0] * (G.a[f][0] - P0[0]) + nv[1] * (G.a[f][1] - P0[1]) + nv[2] * (G.a[f][2] - P0[2]);
            if (to_f > 0.0) { nv[0] = -nv[0]; nv[1] = -nv[1]; nv[2] = -nv[2]; }
            const double nlen = sqrt(nv[0] * nv[0] + nv[1] * nv[1] + nv[2] * nv[2]);
            const double nz = clamp_nz(nv[2], nlen);
            const double inz = 1.0 / nz;
            const double A = -nv[0] * inz, B = -nv[1] * inz;
            pA[f] = A;
            pB[f] = B;
            pD[f] = P0[2] - A * P0[0] - B * P0[1] + A * ox + B * oy;
            if (nz > 0.0) up[nu++] = f; else lo[nl++] = f;
        }
        // an empty side cannot occur for a bounded primitive; guard anyway
        if (nu == 0) { up[nu++] = lo[--nl]; }
        if (nl == 0) { lo[nl++] = up[--nu]; }
        int fmap = 0;
        for (int s = 0; s < 3; ++s) {
            const int fu = up[s < nu ? s : nu - 1];
            const int fl = lo[s < nl ? s : nl - 1];
            out[R_PLANES + 3 * s + 0] = (float)pA[fu];
            out[R_PLANES + 3 * s + 1] = (float)pB[fu];
            out[R_PLANES + 3 * s + 2] = (float)pD[fu];
            out[R_PLANES + 9 + 3 * s + 0] = (float)pA[fl];
            out[R_PLANES + 9 + 3 * s + 1] = (float)pB[fl];
            out[R_PLANES + 9 + 3 * s + 2] = (float)pD[fl];
            fmap |= fu << (2 * s);
            fmap |= fl << (2 * (s + 3));
        }
        out[R_FACEMAP] = __int_as_float(fmap);
    }
    float4* dst = reinterpret_cast<float4*>(rec);
    for (int k = 0; k < kRecordWords / 4; ++k)
        dst[k] = make_float4(out[4 * k], out[4 * k + 1], out[4 * k + 2], out[4 * k + 3]);
    return true;
}

// The colour of a visible slot: SH along the viewing direction (degree
// DEG), written into the record's colour words.
template <int DEG>
__device__ inline void preprocess_colour(const float* shv, const float* mu, const ViewInfo& V,
                                         float* __restrict__ rec) {
    double dx = (double)mu[0] - V.cam_pos[0];
    double dy = (double)mu[1] - V.cam_pos[1];
    double dz = (double)mu[2] - V.cam_pos[2];
    const double idn = 1.0 / sqrt(dx * dx + dy * dy + dz * dz);
    dx *= idn; dy *= idn; dz *= idn;
    constexpr int K = (DEG + 1) * (DEG + 1);
    float Y[16];
    sh_eval_f<DEG>((float)dx, (float)dy, (float)dz, Y);
    float rgb[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        float acc = 0.0f;
#pragma unroll
        for (int k = 0; k < K; ++k) acc = __builtin_fmaf(shv[3 * k + c], Y[k], acc);
        rgb[c] = fmaxf(acc + 0.5f, 0.0f);
    }
    static_assert(R_RGB % 2 == 1, "g, b share an aligned float2");
    rec[R_RGB] = rgb[0];
    *reinterpret_cast<float2*>(rec + R_RGB + 1) = make_float2(rgb[1], rgb[2]);
}

// One thread per primitive, looping over the views: the inputs, the
// rotation, the world-space offsets, sigma and the SH coefficients are
// taken once; per view the thread writes the 32-dword payload record, the
// depth key and the tile count of slot v * n + i.
template <int KIND, int DEG, bool EXACT, bool BYVAL>
__global__ __launch_bounds__(256) void k_preprocess(const float* __restrict__ means, const float* __restrict__ quats,
                                                    const float* __restrict__ dists, const float* __restrict__ opacity,
                                                    const float* __restrict__ sh, int64_t n,
                                                    const ViewInfo* __restrict__ views, int n_views, int tile_shift,
                                                    int aa, float* __restrict__ payload,
                                                    uint32_t* __restrict__ depth_keys, uint32_t* __restrict__ tiles,
                                                    uint2* __restrict__ trect, ViewChunk chunk) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    // BYVAL: the views (at most kViewChunk) come by value; the kernels after
    // this one read them from the workspace, where the first block stores them
    if (BYVAL && blockIdx.x == 0 && threadIdx.x < n_views)
        const_cast<ViewInfo*>(views)[threadIdx.x] = chunk.v[threadIdx.x];
    if (i >= n) return;
    constexpr int nd = (KIND == LINPRIM_OCTAHEDRON) ? 3 : 4;
    float mu[3], qv[4], dv[nd];
#pragma unroll
    for (int c = 0; c < 3; ++c) mu[c] = means[3 * i + c];
#pragma unroll
    for (int c = 0; c < 4; ++c) qv[c] = quats[4 * i + c];
#pragma unroll
    for (int c = 0; c < nd; ++c) dv[c] = dists[nd * i + c];
    const float alpha = opacity[i];
    Geom G;
    const bool ok = build_world(KIND, mu, qv, dv, alpha, G);
    // Eq. 1 density
    double dmin = (double)dv[0];
    for (int k = 1; k < nd; ++k) dmin = fmin(dmin, (double)dv[k]);
    const double sigma = -log(1.0 - kAlphaScaleD * (double)alpha) / (2.0 * dmin);
    // views in chunks of 64: the geometry of every view, then, if the
    // primitive is visible in any, its SH loaded once and the colours
    for (int v0 = 0; v0 < n_views; v0 += 64) {
        const int v1 = min(n_views, v0 + 64);
        uint64_t seen = 0;
        for (int v = v0; v < v1; ++v)
            if (preprocess_view<KIND, EXACT>(ok, G, mu, sigma, BYVAL ? chunk.v[v] : views[v], (int64_t)v * n + i,
                                             tile_shift, aa, payload, depth_keys, tiles, trect))
                seen |= 1ull << (v - v0);
        if (seen) {
            float shv[48];
            load_sh<DEG>(sh + i * (DEG + 1) * (DEG + 1) * 3, shv);
            while (seen) {
                const int v = v0 + __builtin_ctzll(seen);
                seen &= seen - 1;
                preprocess_colour<DEG>(shv, mu, BYVAL ? chunk.v[v] : views[v],
                                       payload + ((int64_t)v * n + i) * kRecordWords);
            }
        }
    }
}
hipError_t launch_preprocess(const linprim_prims& p, int32_t n_views, int tile, bool exact, bool aa,
                             const ViewLayout& L, char* ws, hipStream_t stream, const linprim_camera* cams) {
    // cams != nullptr: the views are not in the workspace yet; up to
    // kViewChunk of them travel with the launch, more are stored first
    ViewChunk chunk;
    int by_value = 0;
    if (cams) {
        if (n_views <= kViewChunk && p.n > 0) {
            int64_t tile_base = 0, pix_base = 0;
            fill_view_chunk(cams, 0, n_views, tile, tile_base, pix_base, chunk);
            by_value = 1;
        } else if (hipError_t e = launch_store_views(cams, n_views, tile, reinterpret_cast<ViewInfo*>(ws + L.views),
                                                     stream)) {
            return e;
        }
    }
    if (p.n == 0) return hipSuccess;
    const int shift = (tile == 8) ? 3 : (tile == 16) ? 4 : 5;
    dim3 grid((unsigned)((p.n + 255) / 256));
    const ViewInfo* views = reinterpret_cast<const ViewInfo*>(ws + L.views);
    float* payload = reinterpret_cast<float*>(ws + L.payload);
    uint32_t* keys = reinterpret_cast<uint32_t*>(ws + L.depth_keys);
    uint32_t* tiles = reinterpret_cast<uint32_t*>(ws + L.tiles);
    uint2* trect = reinterpret_cast<uint2*>(ws + L.trect);
#define LP_PRE_K(K_, D_, E_, B_)                                                                            \
    hipLaunchKernelGGL((k_preprocess<K_, D_, E_, B_>), grid, dim3(256), 0, stream, p.means, p.quats, p.dists,   \
                       p.opacity, p.sh, p.n, views, n_views, shift, aa ? 1 : 0, payload, keys, tiles, trect, chunk)
#define LP_PRE(K_, D_)                                                                                     \
    do {                                                                                                     \
        if (exact) {                                                                                         \
            if (by_value) LP_PRE_K(K_, D_, true, true); else LP_PRE_K(K_, D_, true, false);                \
        } else {                                                                                             \
            if (by_value) LP_PRE_K(K_, D_, false, true); else LP_PRE_K(K_, D_, false, false);              \
        }                                                                                                    \
    } while (0)
#define LP_PRE_DEG(K_)                      \
    switch (p.sh_degree) {                  \
        case 0: LP_PRE(K_, 0); break;       \
        case 1: LP_PRE(K_, 1); break;       \
        case 2: LP_PRE(K_, 2); break;       \
        default: LP_PRE(K_, 3); break;      \
    }
    if (p.type == LINPRIM_OCTAHEDRON) {
        LP_PRE_DEG(LINPRIM_OCTAHEDRON)
    } else {
        LP_PRE_DEG(LINPRIM_TETRAHEDRON)
    }
#undef LP_PRE_DEG
#undef LP_PRE
#undef LP_PRE_K
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Exclusive prefix sum of the tile counts (two passes: block totals, then
// block-local scans, each block adding the totals of the blocks before it;
// beyond kScanDirectBlocks blocks a single-block prefix of the totals runs
// in between).
// ---------------------------------------------------------------------------
__device__ inline uint64_t block_exclusive_scan_u64(uint64_t x, uint64_t* lds, uint64_t* total) {
    // 256 threads: Hillis-Steele in shared memory
    const int t = threadIdx.x;
    lds[t] = x;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
        const uint64_t y = (t >= off) ? lds[t - off] : 0;
        __syncthreads();
        lds[t] += y;
        __syncthreads();
    }
    const uint64_t incl = lds[t];
    *total = lds[255];
    __syncthreads();
    return incl - x;
}

// Per block of kScanItems slots: the sum of the tile counts and the number
// of slots that touch a tile (block_sums[b] and vis_sums[b]).
// The status of an empty slot range (no primitives).
__global__ void k_status_empty(Status* __restrict__ status) {
    if (threadIdx.x == 0) {
        status->n_pairs = 0;
        status->n_vis = 0;
        status->overflow = 0;
        status->n_big = 0;
        status->n_mid = 0;
        status->n_huge = 0;
    }
}

__global__ __launch_bounds__(256) void k_scan_reduce(const uint32_t* __restrict__ in, int64_t count,
                                                     uint64_t* __restrict__ block_sums,
                                                     uint64_t* __restrict__ vis_sums, Status* __restrict__ status) {
    // the lists k_scan_apply appends to start empty
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        status->overflow = 0;
        status->n_big = 0;
        status->n_mid = 0;
        status->n_huge = 0;
    }
    __shared__ uint64_t part[2][4];
    const int64_t base = (int64_t)blockIdx.x * kScanItems;
    uint64_t s = 0, c = 0;
    for (int k = 0; k < kScanItems / 256; ++k) {
        const int64_t idx = base + k * 256 + threadIdx.x;
        const uint32_t x = (idx < count) ? in[idx] : 0u;
        s += x;
        c += x ? 1u : 0u;
    }
    for (int off = 32; off >= 1; off >>= 1) {
        s += __shfl_xor(s, off, 64);
        c += __shfl_xor(c, off, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        part[0][threadIdx.x >> 6] = s;
        part[1][threadIdx.x >> 6] = c;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        block_sums[blockIdx.x] = part[0][0] + part[0][1] + part[0][2] + part[0][3];
        vis_sums[blockIdx.x] = part[1][0] + part[1][1] + part[1][2] + part[1][3];
    }
}

// Many blocks (k_scan_apply would re-add too many block totals): one block
// turns the block totals into exclusive prefixes first, in place.
__global__ __launch_bounds__(256) void k_scan_prefix(uint64_t* __restrict__ block_sums,
                                                     uint64_t* __restrict__ vis_sums, int64_t nblocks,
                                                     Status* __restrict__ status) {
    __shared__ uint64_t lds[256];
    uint64_t carry = 0, vcarry = 0;
    for (int64_t b0 = 0; b0 < nblocks; b0 += 256) {
        const int64_t idx = b0 + threadIdx.x;
        const uint64_t x = (idx < nblocks) ? block_sums[idx] : 0;
        const uint64_t y = (idx < nblocks) ? vis_sums[idx] : 0;
        uint64_t total, vtotal;
        const uint64_t ex = block_exclusive_scan_u64(x, lds, &total);
        const uint64_t vex = block_exclusive_scan_u64(y, lds, &vtotal);
        if (idx < nblocks) {
            block_sums[idx] = carry + ex;
            vis_sums[idx] = vcarry + vex;
        }
        carry += total;
        vcarry += vtotal;
    }
    if (threadIdx.x == 0) {
        status->n_pairs = carry;
        status->n_vis = (uint32_t)vcarry;
    }
}

// Sum of x[0, count) over the block (every thread gets it).
__device__ inline uint64_t block_sum_u64(const uint64_t* __restrict__ x, int64_t count, uint64_t* part4) {
    uint64_t s = 0;
    for (int64_t b = threadIdx.x; b < count; b += blockDim.x) s += x[b];
    for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off, 64);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) part4[threadIdx.x >> 6] = s;
    __syncthreads();
    return part4[0] + part4[1] + part4[2] + part4[3];
}

// Appends a slot to a list (in no particular order) with one atomic per
// wave and item.
__device__ inline void wave_append(bool take, uint32_t value, uint32_t* __restrict__ counter,
                                   uint32_t* __restrict__ list, int lane, uint64_t lt_mask) {
    const uint64_t m = __ballot(take);
    if (!m) return;
    const int leader = __builtin_ctzll(m);
    uint32_t first = 0;
    if (lane == leader) first = atomicAdd(counter, (uint32_t)__popcll(m));
    first = __shfl(first, leader, 64);
    if (take) list[first + __popcll(m & lt_mask)] = value;
}

// Exclusive scan of two counters over the 256 threads of a block (wave
// shuffles, then the four wave totals); a and b become the sums over the
// threads before this one, ta and tb the block totals.
__device__ inline void block_scan2_u64(uint64_t& a, uint64_t& b, uint64_t* part8, uint64_t& ta, uint64_t& tb) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    uint64_t ia = a, ib = b;
    for (int off = 1; off < 64; off <<= 1) {
        const uint64_t ya = __shfl_up(ia, off, 64), yb = __shfl_up(ib, off, 64);
        if (lane >= off) {
            ia += ya;
            ib += yb;
        }
    }
    if (lane == 63) {
        part8[w] = ia;
        part8[4 + w] = ib;
    }
    __syncthreads();
    uint64_t pa = 0, pb = 0;
    for (int k = 0; k < 4; ++k)
        if (k < w) {
            pa += part8[k];
            pb += part8[4 + k];
        }
    ta = part8[0] + part8[1] + part8[2] + part8[3];
    tb = part8[4] + part8[5] + part8[6] + part8[7];
    a = pa + ia - a;
    b = pb + ib - b;
}

// Also lists, in slot order, the slots that touch a tile (for the
// preprocessing backward), and, in no particular order, those with more than
// kBigRun gradient records (tile count x groups per tile) up to kHugeRun
// tiles and those with more than kHugeRun tiles; per block in slot order, the slots with more
// than kMidRun up to kBigRun records (the mid list, from the end of the big
// list's array).  The block's counts are loaded and its offsets
// and list entries stored coalesced, through LDS; each thread scans 16
// consecutive slots in between.
__global__ __launch_bounds__(256) void k_scan_apply(const uint32_t* __restrict__ in, int64_t count,
                                                    const uint64_t* __restrict__ block_sums,
                                                    const uint64_t* __restrict__ vis_sums, int64_t nblocks,
                                                    bool prefixed, uint32_t* __restrict__ out, int nq,
                                                    Status* __restrict__ status, uint32_t* __restrict__ big,
                                                    uint32_t* __restrict__ vis, uint32_t* __restrict__ huge) {
    constexpr int PER = kScanItems / 256;
    // slot e of the block at e + e / PER: a thread's PER consecutive slots
    // then fall in distinct banks across the wave
    __shared__ uint32_t stage[kScanItems + kScanItems / PER];
    __shared__ uint32_t vstage[kScanItems];
    __shared__ uint64_t part4[4];
    __shared__ uint64_t part8[8];
    // this block's start: the sums of the blocks before it (a few hundred
    // values for a million slots), or the prefix k_scan_prefix wrote
    uint64_t pre, vpre;
    if (prefixed) {
        pre = block_sums[blockIdx.x];
        vpre = vis_sums[blockIdx.x];
    } else {
        pre = block_sum_u64(block_sums, blockIdx.x, part4);
        vpre = block_sum_u64(vis_sums, blockIdx.x, part4);
        if (blockIdx.x == nblocks - 1 && threadIdx.x == 0) {
            status->n_pairs = pre + block_sums[blockIdx.x];
            status->n_vis = (uint32_t)(vpre + vis_sums[blockIdx.x]);
        }
    }
    const int t = threadIdx.x;
    const int64_t base = (int64_t)blockIdx.x * kScanItems;
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        const int e = k * 256 + t;
        const int64_t idx = base + e;
        stage[e + e / PER] = (idx < count) ? in[idx] : 0u;
    }
    __syncthreads();
    uint32_t v[PER];
    // per thread: tile sum; slots that touch a tile (low word) and mid slots
    // (high word), scanned together
    uint64_t s = 0, c = 0;
    auto is_mid = [nq](uint32_t x) {
        const int64_t nrec = (int64_t)x * nq;
        return nrec > kMidRun && nrec <= kBigRun;
    };
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        v[k] = stage[t * (PER + 1) + k];
        s += v[k];
        c += (v[k] ? 1u : 0u) + (is_mid(v[k]) ? (1ull << 32) : 0ull);
    }
    uint64_t ts, tc;
    block_scan2_u64(s, c, part8, ts, tc);
    // the block's mid slots take one run of the mid list (a single atomic)
    __shared__ uint32_t mid_base;
    if (t == 0 && (tc >> 32)) mid_base = atomicAdd(&status->n_mid, (uint32_t)(tc >> 32));
    uint64_t run = pre + s;
    uint32_t lv = (uint32_t)c, lm = (uint32_t)(c >> 32);
    const int lane = t & 63;
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        const uint32_t idx = (uint32_t)(base + (int64_t)t * PER + k);
        stage[t * (PER + 1) + k] = (uint32_t)run;
        run += v[k];
        if (v[k]) vstage[lv++] = idx;
        // (slots over kHugeRun tiles are on the huge list, which also serves
        // their record sums)
        wave_append((int64_t)v[k] * nq > kBigRun && v[k] <= (uint32_t)kHugeRun, idx, &status->n_big, big, lane, lt_mask);
        wave_append(v[k] > (uint32_t)kHugeRun, idx, &status->n_huge, huge, lane, lt_mask);
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        const int e = k * 256 + t;
        const int64_t idx = base + e;
        if (idx < count) out[idx] = stage[e + e / PER];
        const int64_t own = base + (int64_t)t * PER + k;
        if (is_mid(v[k])) big[count - 1 - (int64_t)(mid_base + lm++)] = (uint32_t)own;
    }
    for (int j = t; j < (int)(uint32_t)tc; j += 256) vis[vpre + j] = vstage[j];
}

hipError_t launch_scan(const ViewLayout& L, char* ws, int tile, hipStream_t stream) {
    const int64_t count = L.n * L.n_views;
    const uint32_t* tiles = reinterpret_cast<const uint32_t*>(ws + L.tiles);
    uint32_t* offsets = reinterpret_cast<uint32_t*>(ws + L.offsets);
    uint64_t* bsums = reinterpret_cast<uint64_t*>(ws + L.block_sums);
    Status* status = reinterpret_cast<Status*>(ws + L.status);
    uint32_t* big = reinterpret_cast<uint32_t*>(ws + L.big);
    const int nq = (tile / 8) * (tile / 8);
    const int64_t nb = L.scan_blocks;
    uint64_t* vsums = bsums + (nb + 1);
    if (nb > 0) {
        hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)nb), dim3(256), 0, stream, tiles, count, bsums, vsums, status);
        const bool prefixed = nb > kScanDirectBlocks;
        if (prefixed) hipLaunchKernelGGL(k_scan_prefix, dim3(1), dim3(256), 0, stream, bsums, vsums, nb, status);
        hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)nb), dim3(256), 0, stream, tiles, count, bsums, vsums, nb,
                           prefixed, offsets, nq, status, big, reinterpret_cast<uint32_t*>(ws + L.vis),
                           reinterpret_cast<uint32_t*>(ws + L.huge));
    } else {
        hipLaunchKernelGGL(k_status_empty, dim3(1), dim3(64), 0, stream, status);
    }
    return hipGetLastError();
}

}  // namespace linprim
