// k_prep_bwd.hip -- preprocessing backward pass (Sec. 3.4 "Preprocessing
// Backpropagation"): per primitive, sum its per-tile gradient records, then
// undo the plane construction, the ray-space projection and the view
// transform, and split the corner gradients onto rotation and distances.
// One thread per primitive loops over the views, so gradients summed over
// views are deterministic.  Geometry in double precision (memory-bound).
#include "linprim_common.h"

namespace linprim {

__device__ inline void cross3(const double a[3], const double b[3], double o[3]) {
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
}

// Record r of a primitive (tile r / NQ of its tile rectangle in row-major
// order, group r % NQ of that tile) exists only if the group meets the
// primitive's pixel rectangle.
__device__ inline bool record_exists(int r, int NQ, int QX, int tile, int4 rect, int tx0, int ty0, int ntx) {
    const int t = r / NQ, q = r % NQ;
    const int tx = tx0 + t % ntx, ty = ty0 + t / ntx;
    const int gx0 = tx * tile + (q % QX) * 8, gy0 = ty * tile + (q / QX) * 8;
    return !(rect.x > gx0 + 7 || rect.z < gx0 || rect.y > gy0 + 7 || rect.w < gy0);
}

// Sums the gradient records of the slots with more than kMidRun records.
// The run of a slot with more than kBigRun records is cut into kBigChunks
// equal chunks; for a huge slot (more than kHugeRun tiles) one wavefront per
// chunk strides over it, sums across lanes in a fixed order and writes the
// chunk's sum into the chunk's first record, so no wave holds up the kernel
// with a long run and the result does not depend on scheduling.  k_slot_bwd
// adds the chunk sums in chunk order; shorter runs it sums itself.
__device__ inline void sum_big_chunk(const float* __restrict__ payload, const uint32_t* __restrict__ tiles,
                                     const uint32_t* __restrict__ offsets, int64_t slot, int c, int tile,
                                     float* __restrict__ grads, int lane) {
    const int QX = tile / 8, NQ = QX * QX;
    const int shift = (tile == 8) ? 3 : (tile == 16) ? 4 : 5;
    const int nr = (int)tiles[slot] * NQ;
    const int r0 = big_chunk_start(c, nr), r1 = big_chunk_start(c + 1, nr);
    const uint32_t o = offsets[slot];
    // the pixel rectangle decides which records exist only with several
    // groups per tile
    const int4 rc = (NQ == 1) ? make_int4(0, 0, 0, 0) : *reinterpret_cast<const int4*>(payload + slot * kRecordWords);
    const int tx0 = rc.x >> shift, ty0 = rc.y >> shift, ntx = (rc.z >> shift) - tx0 + 1;
    float acc[kGradWords];
#pragma unroll
    for (int k = 0; k < kGradWords; ++k) acc[k] = 0.0f;
    const float4* g = reinterpret_cast<const float4*>(grads + (int64_t)o * NQ * kGradWords);
    for (int rb = r0 + lane; rb < r1; rb += 256) {
        // four records per lane per iteration, all twenty loads in flight
        // together (the longest chunk bounds the kernel's time)
        float4 x[4][kGradWords / 4];
        bool use[4];
#pragma unroll
        for (int h = 0; h < 4; ++h) {
            const int r = rb + 64 * h;
            use[h] = r < r1 && (NQ == 1 || record_exists(r, NQ, QX, tile, rc, tx0, ty0, ntx));
#pragma unroll
            for (int k = 0; k < kGradWords / 4; ++k)
                x[h][k] = use[h] ? g[(int64_t)r * (kGradWords / 4) + k] : make_float4(0.f, 0.f, 0.f, 0.f);
        }
#pragma unroll
        for (int h = 0; h < 4; ++h)
#pragma unroll
            for (int k = 0; k < kGradWords / 4; ++k) {
                acc[4 * k] += x[h][k].x;
                acc[4 * k + 1] += x[h][k].y;
                acc[4 * k + 2] += x[h][k].z;
                acc[4 * k + 3] += x[h][k].w;
            }
    }
    const float outv = wave_reduce20(acc, lane);
    const int ridx = reduce20_index(lane);
    if (ridx >= 0) grads[((int64_t)o * NQ + r0) * kGradWords + ridx] = outv;
}

// A mid slot's run (kMidRun < records <= kBigRun) summed by twenty lanes, one
// word each, in record order: the same additions, in the same order, as the
// slot's own thread in k_slot_bwd makes for a short run.  The sum goes into
// the slot's first record, once every lane of the slot has read it.
__device__ inline void sum_mid_slot(const float* __restrict__ payload, const uint32_t* __restrict__ tiles,
                                    const uint32_t* __restrict__ offsets, int64_t slot, int w, int tile,
                                    float* __restrict__ grads) {
    const int QX = tile / 8, NQ = QX * QX;
    const int shift = (tile == 8) ? 3 : (tile == 16) ? 4 : 5;
    const int nr = (int)tiles[slot] * NQ;
    const uint32_t o = offsets[slot];
    // the pixel rectangle decides which records exist only with several
    // groups per tile
    const int4 rc = (NQ == 1) ? make_int4(0, 0, 0, 0) : *reinterpret_cast<const int4*>(payload + slot * kRecordWords);
    const int tx0 = rc.x >> shift, ty0 = rc.y >> shift, ntx = (rc.z >> shift) - tx0 + 1;
    float* g = grads + (int64_t)o * NQ * kGradWords + w;
    float acc = 0.0f;
    constexpr int B = 16;
    for (int q0 = 0; q0 < nr; q0 += B) {
        float x[B];
#pragma unroll
        for (int h = 0; h < B; ++h) {
            const int q = q0 + h;
            const bool use = q < nr && (NQ == 1 || record_exists(q, NQ, QX, tile, rc, tx0, ty0, ntx));
            x[h] = use ? g[(int64_t)q * kGradWords] : 0.0f;
        }
#pragma unroll
        for (int h = 0; h < B; ++h) acc += x[h];
    }
    g[0] = acc;
}

// A big slot's run (more than kBigRun records, up to kHugeRun tiles) summed
// by one wave: four lanes per chunk (lane l takes chunk l / 4), each lane the
// chunk's records l % 4, l % 4 + 4, ... in order, four loads in flight, then
// the four lanes' sums added across the quad; the quad's first lane writes
// the chunk's sum into the chunk's first record.
__device__ inline void sum_big_quads(const float* __restrict__ payload, const uint32_t* __restrict__ tiles,
                                     const uint32_t* __restrict__ offsets, int64_t slot, int tile,
                                     float* __restrict__ grads, int lane) {
    const int QX = tile / 8, NQ = QX * QX;
    const int shift = (tile == 8) ? 3 : (tile == 16) ? 4 : 5;
    const int nr = (int)tiles[slot] * NQ;
    const int c = lane >> 2, sub = lane & 3;
    const int r0 = big_chunk_start(c, nr), r1 = big_chunk_start(c + 1, nr);
    const uint32_t o = offsets[slot];
    const int4 rc = (NQ == 1) ? make_int4(0, 0, 0, 0) : *reinterpret_cast<const int4*>(payload + slot * kRecordWords);
    const int tx0 = rc.x >> shift, ty0 = rc.y >> shift, ntx = (rc.z >> shift) - tx0 + 1;
    float acc[kGradWords];
#pragma unroll
    for (int k = 0; k < kGradWords; ++k) acc[k] = 0.0f;
    const float4* g = reinterpret_cast<const float4*>(grads + (int64_t)o * NQ * kGradWords);
    for (int rb = r0 + sub; rb < r1; rb += 16) {
        float4 x[4][kGradWords / 4];
#pragma unroll
        for (int h = 0; h < 4; ++h) {
            const int r = rb + 4 * h;
            const bool use = r < r1 && (NQ == 1 || record_exists(r, NQ, QX, tile, rc, tx0, ty0, ntx));
#pragma unroll
            for (int k = 0; k < kGradWords / 4; ++k)
                x[h][k] = use ? g[(int64_t)r * (kGradWords / 4) + k] : make_float4(0.f, 0.f, 0.f, 0.f);
        }
#pragma unroll
        for (int h = 0; h < 4; ++h)
#pragma unroll
            for (int k = 0; k < kGradWords / 4; ++k) {
                acc[4 * k] += x[h][k].x;
                acc[4 * k + 1] += x[h][k].y;
                acc[4 * k + 2] += x[h][k].z;
                acc[4 * k + 3] += x[h][k].w;
            }
    }
    // quad sums: lanes i and i ^ 1, then i and i ^ 2
#pragma unroll
    for (int k = 0; k < kGradWords; ++k) {
        acc[k] += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(acc[k]), 0xB1, 0xF, 0xF, false));
        acc[k] += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(acc[k]), 0x4E, 0xF, 0xF, false));
    }
    if (sub == 0) {
        float4* dst = reinterpret_cast<float4*>(grads + ((int64_t)o * NQ + r0) * kGradWords);
#pragma unroll
        for (int k = 0; k < kGradWords / 4; ++k)
            dst[k] = make_float4(acc[4 * k], acc[4 * k + 1], acc[4 * k + 2], acc[4 * k + 3]);
    }
}

constexpr int kMidPerWave = 64 / kGradWords;   // mid slots per wavefront (three)

// Items: kBigChunks per huge slot (one wave per chunk), one per big slot
// (sum_big_quads), one per kMidPerWave mid slots.
__global__ __launch_bounds__(256) void k_sum_big(const float* __restrict__ payload,
                                                 const uint32_t* __restrict__ tiles,
                                                 const uint32_t* __restrict__ offsets,
                                                 const uint32_t* __restrict__ big,
                                                 const uint32_t* __restrict__ huge, int64_t n_slots, int tile,
                                                 const Status* __restrict__ status, uint64_t capacity,
                                                 float* __restrict__ grads) {
    if (status->n_pairs > capacity) return;
    const int lane = threadIdx.x & 63;
    const int64_t waves = (int64_t)gridDim.x * (blockDim.x >> 6);
    const int64_t n_chunked = (int64_t)status->n_huge * kBigChunks;
    const int64_t n_quads = n_chunked + status->n_big;
    const int64_t n_mid = status->n_mid;
    const int64_t items = n_quads + (n_mid + kMidPerWave - 1) / kMidPerWave;
    for (int64_t it = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); it < items; it += waves) {
        if (it < n_chunked) {
            sum_big_chunk(payload, tiles, offsets, huge[it / kBigChunks], (int)(it % kBigChunks), tile, grads, lane);
        } else if (it < n_quads) {
            sum_big_quads(payload, tiles, offsets, big[it - n_chunked], tile, grads, lane);
        } else {
            const int64_t m = (it - n_quads) * kMidPerWave + lane / kGradWords;
            if (lane < kMidPerWave * kGradWords && m < n_mid)
                sum_mid_slot(payload, tiles, offsets, big[n_slots - 1 - m], lane % kGradWords, tile, grads);
        }
    }
}

// Colour backward along the viewing direction, one basis function at a
// time (single precision): gsh_k += grgb Y_k, gdir += sum_ch grgb sh_k
// dY_k/ddir.  The basis polynomials are those of sh_eval_f.
struct ShBack {
    int K;
    const float* sh;     // [48] coefficients (registers)
    float* gsh;          // [48] accumulators
    float gr[3];
    float gdir[3];
    __device__ inline void term(int k, float Y, float gx, float gy, float gz) {
        if (k >= K) return;
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) {
            gsh[3 * k + ch] += gr[ch] * Y;
            const float w = gr[ch] * sh[3 * k + ch];
            gdir[0] += w * gx;
            gdir[1] += w * gy;
            gdir[2] += w * gz;
        }
    }
};

// The same terms with the coefficient gradients added to an LDS row:
// coefficient word w of this thread at acc[w * stride] (coefficient-major,
// so that the lanes of a wave add to consecutive banks).
struct ShLds {
    int K;
    const float* sh;     // [48] coefficients (registers)
    float* acc;          // this thread's column of the block's LDS stage
    int stride;
    float gr[3];
    float gdir[3];
    __device__ inline void term(int k, float Y, float gx, float gy, float gz) {
        if (k >= K) return;
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) {
            acc[(3 * k + ch) * stride] += gr[ch] * Y;
            const float w = gr[ch] * sh[3 * k + ch];
            gdir[0] += w * gx;
            gdir[1] += w * gy;
            gdir[2] += w * gz;
        }
    }
};

// The same terms with the coefficient gradients stored as they are made
// (one view: no accumulation over views), so that they need no registers.
struct ShStore {
    int K;
    const float* sh;     // [48] coefficients (registers)
    float* gs;           // the primitive's row of dL/dSH (global)
    float gr[3];
    float gdir[3];
    __device__ inline void term(int k, float Y, float gx, float gy, float gz) {
        if (k >= K) return;
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) {
            gs[3 * k + ch] = gr[ch] * Y;
            const float w = gr[ch] * sh[3 * k + ch];
            gdir[0] += w * gx;
            gdir[1] += w * gy;
            gdir[2] += w * gz;
        }
    }
};

struct ShConstF {
    float c0, c1, c2a, c2b, c2c, c3a, c3b, c3c, c3d, c3e;
};

__device__ inline ShConstF sh_constants_f() {
    const ShConst K = sh_constants();
    return {(float)K.c0, (float)K.c1, (float)K.c2a, (float)K.c2b, (float)K.c2c,
            (float)K.c3a, (float)K.c3b, (float)K.c3c, (float)K.c3d, (float)K.c3e};
}

// raw colour (before the clamp) along dir, single precision
__device__ inline void sh_raw_f(int K, const float* sh, float x, float y, float z, float raw[3]) {
    const ShConstF C = sh_constants_f();
    float Y[16];
    Y[0] = C.c0;
    Y[1] = -C.c1 * y; Y[2] = C.c1 * z; Y[3] = -C.c1 * x;
    Y[4] = C.c2a * x * y; Y[5] = -C.c2a * y * z; Y[6] = C.c2b * (2 * z * z - x * x - y * y);
    Y[7] = -C.c2a * x * z; Y[8] = C.c2c * (x * x - y * y);
    Y[9] = -C.c3a * y * (3 * x * x - y * y); Y[10] = C.c3b * x * y * z;
    Y[11] = -C.c3c * y * (4 * z * z - x * x - y * y); Y[12] = C.c3d * z * (2 * z * z - 3 * x * x - 3 * y * y);
    Y[13] = -C.c3c * x * (4 * z * z - x * x - y * y); Y[14] = C.c3e * z * (x * x - y * y);
    Y[15] = -C.c3a * x * (x * x - 3 * y * y);
    raw[0] = raw[1] = raw[2] = 0.5f;
#pragma unroll
    for (int k = 0; k < 16; ++k)
        if (k < K)
            for (int ch = 0; ch < 3; ++ch) raw[ch] += sh[3 * k + ch] * Y[k];
}

template <class S_>
__device__ inline void sh_backward(S_& S, float x, float y, float z) {
    const ShConstF K = sh_constants_f();
    S.term(0, K.c0, 0, 0, 0);
    S.term(1, -K.c1 * y, 0, -K.c1, 0);
    S.term(2, K.c1 * z, 0, 0, K.c1);
    S.term(3, -K.c1 * x, -K.c1, 0, 0);
    S.term(4, K.c2a * x * y, K.c2a * y, K.c2a * x, 0);
    S.term(5, -K.c2a * y * z, 0, -K.c2a * z, -K.c2a * y);
    S.term(6, K.c2b * (2 * z * z - x * x - y * y), -2 * K.c2b * x, -2 * K.c2b * y, 4 * K.c2b * z);
    S.term(7, -K.c2a * x * z, -K.c2a * z, 0, -K.c2a * x);
    S.term(8, K.c2c * (x * x - y * y), 2 * K.c2c * x, -2 * K.c2c * y, 0);
    S.term(9, -K.c3a * y * (3 * x * x - y * y), -6 * K.c3a * x * y, -K.c3a * (3 * x * x - 3 * y * y), 0);
    S.term(10, K.c3b * x * y * z, K.c3b * y * z, K.c3b * x * z, K.c3b * x * y);
    S.term(11, -K.c3c * y * (4 * z * z - x * x - y * y), 2 * K.c3c * x * y, -K.c3c * (4 * z * z - x * x - 3 * y * y),
           -8 * K.c3c * y * z);
    S.term(12, K.c3d * z * (2 * z * z - 3 * x * x - 3 * y * y), -6 * K.c3d * x * z, -6 * K.c3d * y * z,
           K.c3d * (6 * z * z - 3 * x * x - 3 * y * y));
    S.term(13, -K.c3c * x * (4 * z * z - x * x - y * y), -K.c3c * (4 * z * z - 3 * x * x - y * y), 2 * K.c3c * x * y,
           -8 * K.c3c * x * z);
    S.term(14, K.c3e * z * (x * x - y * y), 2 * K.c3e * x * z, -2 * K.c3e * y * z, K.c3e * (x * x - y * y));
    S.term(15, -K.c3a * x * (x * x - 3 * y * y), -K.c3a * (3 * x * x - 3 * y * y), 6 * K.c3a * x * y, 0);
}

// Offsets of one primitive (camera space) -> world offsets -> rotation
// gradient (row-major) and distance gradients, accumulated.
template <int KIND>
__device__ inline void offsets_to_rotation(const Geom& G, const ViewInfo& V, const float* __restrict__ dists,
                                          const double goc[4][3], double gR[9], double gd[4]) {
    constexpr int ND = (KIND == LINPRIM_OCTAHEDRON) ? 3 : 4;
#pragma unroll
    for (int k = 0; k < ND; ++k) {
        double go[3];
        for (int c = 0; c < 3; ++c) go[c] = V.Rw[c] * goc[k][0] + V.Rw[3 + c] * goc[k][1] + V.Rw[6 + c] * goc[k][2];
        if (KIND == LINPRIM_OCTAHEDRON) {
            const double dk = (double)dists[k];
            for (int rr = 0; rr < 3; ++rr) {
                gR[3 * rr + k] += go[rr] * dk;
                gd[k] += go[rr] * G.R[3 * rr + k];
            }
        } else {
            const double gk = (double)dists[k] * kInvSqrt3;
            for (int rr = 0; rr < 3; ++rr) {
                const double rb = kTetDir[k][0] * G.R[3 * rr] + kTetDir[k][1] * G.R[3 * rr + 1] +
                                  kTetDir[k][2] * G.R[3 * rr + 2];
                for (int c = 0; c < 3; ++c) gR[3 * rr + c] += go[rr] * kTetDir[k][c] * gk;
                gd[k] += go[rr] * rb * kInvSqrt3;
            }
        }
    }
}

// The slot result, in the layout the record summation leaves it in:
//   [0..2] dL/d mu (geometric part), [3..11] dL/dR (row-major),
//   [12..15] dL/d distances, [16..18] dL/d rgb, [19] dL/d sigma.
__device__ inline void pack_slot_result(const double gm[3], const double gR[9], const double gd[4], float gr, float gg,
                                        float gb, float gsig, float res[kGradWords]) {
    for (int c = 0; c < 3; ++c) res[c] = (float)gm[c];
    for (int c = 0; c < 9; ++c) res[3 + c] = (float)gR[c];
    for (int c = 0; c < 4; ++c) res[12 + c] = (float)gd[c];
    res[16] = gr;
    res[17] = gg;
    res[18] = gb;
    res[19] = gsig;
}

// Exact variant (no ray space): the summed record holds, per plane k,
// dL/d(a_k, b_k) at the rectangle origin (words 0, 1), dL/du_k (word 2, the
// plane's offset g_k = a_k ox + b_k oy) and dL/dc_k (word 3), plus
// dL/d(sigma z_c) (word 19).  With the camera-space normal n_k and centre t:
//   a_k = -t_z n_kx / fx,  b_k = -t_z n_ky / fy,  c_k = n_k . t,
//   ox = i0 + 1/2 - (fx t_x / t_z + cx),  oy likewise,
// then n_k -> camera offsets oc (and, for octahedra, the 1/d^2 weights).
template <int KIND>
__device__ inline void exact_slot_bwd(const Geom& G, const ViewInfo& V, const float* __restrict__ dists, double sigma,
                                      double ox, double oy, const float r[kGradWords], float res[kGradWords]) {
    double nrm[4][3];
    exact_normals(KIND, G, nrm);
    const double tx = G.tc[0], ty = G.tc[1], tz = G.tc[2];
    double gt[3] = {0, 0, 0}, gn[4][3];
    double gox = 0.0, goy = 0.0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const double a = -tz * nrm[k][0] / V.fx, b = -tz * nrm[k][1] / V.fy;
        const double w0 = r[4 * k], w1 = r[4 * k + 1], w2 = r[4 * k + 2], w3 = r[4 * k + 3];
        const double ga = w0 + w2 * ox, gb = w1 + w2 * oy;
        gox += w2 * a;
        goy += w2 * b;
        gn[k][0] = -tz / V.fx * ga + tx * w3;
        gn[k][1] = -tz / V.fy * gb + ty * w3;
        gn[k][2] = tz * w3;
        gt[0] += nrm[k][0] * w3;
        gt[1] += nrm[k][1] * w3;
        gt[2] += nrm[k][2] * w3 - nrm[k][0] / V.fx * ga - nrm[k][1] / V.fy * gb;
    }
    // projected centre: X = fx t_x / t_z + cx, ox = (i0 + i1)/2 + 1/2 - X
    gt[0] -= gox * V.fx / tz;
    gt[2] += gox * V.fx * tx / (tz * tz);
    gt[1] -= goy * V.fy / tz;
    gt[2] += goy * V.fy * ty / (tz * tz);
    // the record's sigma is sigma t_z
    const double gsig = (double)r[19] * tz;
    gt[2] += (double)r[19] * sigma;
    double goc[4][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
    double gd[4] = {0, 0, 0, 0};
    if (KIND == LINPRIM_OCTAHEDRON) {
        // n_k = N^T kSlab[k] with N = M^-1 and column c of M the offset oc_c:
        // dL/dN[c][r] = sum_k kSlab[k][c] dL/dn_k[r], dL/dM = -N^T dL/dN N^T
        double M[9], N[9], gN[9];
        for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 3; ++c) M[3 * r + c] = G.oc[c][r];
        inverse3(M, N);
        for (int c = 0; c < 3; ++c)
            for (int r = 0; r < 3; ++r)
                gN[3 * c + r] = kSlab[0][c] * gn[0][r] + kSlab[1][c] * gn[1][r] + kSlab[2][c] * gn[2][r] +
                                kSlab[3][c] * gn[3][r];
        double T1[9];
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b)
                T1[3 * a + b] = N[a] * gN[b] + N[3 + a] * gN[3 + b] + N[6 + a] * gN[6 + b];
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b)
                goc[b][a] = -(T1[3 * a] * N[3 * b] + T1[3 * a + 1] * N[3 * b + 1] + T1[3 * a + 2] * N[3 * b + 2]);
    } else {
        // rows of M_f are the offsets of the three corners other than f and
        // M_f n_f = 1:  dL/dM_f = -(M_f^-T dL/dn_f) n_f^T
        for (int f = 0; f < 4; ++f) {
            double M[9], N[9];
            int m[3], q = 0;
            for (int kk = 0; kk < 4; ++kk) {
                if (kk == f) continue;
                m[q] = kk;
                for (int c = 0; c < 3; ++c) M[3 * q + c] = G.oc[kk][c];
                ++q;
            }
            inverse3(M, N);
            double y[3];
            for (int j = 0; j < 3; ++j) y[j] = N[j] * gn[f][0] + N[3 + j] * gn[f][1] + N[6 + j] * gn[f][2];
            for (int j = 0; j < 3; ++j)
                for (int c = 0; c < 3; ++c) goc[m[j]][c] -= y[j] * nrm[f][c];
        }
    }
    double gR[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    offsets_to_rotation<KIND>(G, V, dists, goc, gR, gd);
    double gm[3];
    for (int c = 0; c < 3; ++c) gm[c] = V.Rw[c] * gt[0] + V.Rw[3 + c] * gt[1] + V.Rw[6 + c] * gt[2];
    pack_slot_result(gm, gR, gd, r[16], r[17], r[18], (float)gsig, res);
}

// Ray-space variant: the summed record r (dL/d plane coefficients, dL/d rgb,
// dL/d sigma) -> dL/d(ray-space centre, offsets) -> camera -> world, into the
// slot result.  `stat` receives the view-space positional gradient and the
// screen radius used by population control.
template <int KIND>
__device__ inline void ray_slot_bwd(const Geom& G, const ViewInfo& V, const float dv[4], double ox, double oy,
                                    const float r[kGradWords], float res[kGradWords], float2& stat) {
    constexpr int ND = (KIND == LINPRIM_OCTAHEDRON) ? 3 : 4;
    // ---- planes -> ray-space centre (xy) and offsets a_k
    double gox = 0.0, goy = 0.0;
    double ga[4][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
    if (KIND == LINPRIM_OCTAHEDRON) {
        double M[9], N[9], gN[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
        for (int rr = 0; rr < 3; ++rr)
            for (int k = 0; k < 3; ++k) M[3 * rr + k] = G.a[k][rr];
        inverse3(M, N);
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            double nu[3];
            for (int c = 0; c < 3; ++c) nu[c] = kSlab[s][0] * N[c] + kSlab[s][1] * N[3 + c] + kSlab[s][2] * N[6 + c];
            const double nl = sqrt(nu[0] * nu[0] + nu[1] * nu[1] + nu[2] * nu[2]);
            const double nz = clamp_nz(nu[2], nl);
            const double inz = 1.0 / nz;
            const double A = -nu[0] * inz, B = -nu[1] * inz, Wd = fabs(inz);
            const double gA = r[4 * s], gB = r[4 * s + 1], gUp = r[4 * s + 2], gLo = r[4 * s + 3];
            const double gsum = gUp + gLo;         // both offsets carry A ox + B oy
            const double gW = gUp - gLo;
            const double gAt = gA + gsum * ox, gBt = gB + gsum * oy;
            gox += gsum * A;
            goy += gsum * B;
            const double gn0 = -gAt * inz, gn1 = -gBt * inz, gn2 = -(gAt * A + gBt * B + gW * Wd) * inz;
            for (int q = 0; q < 3; ++q) {
                gN[3 * q + 0] += kSlab[s][q] * gn0;
                gN[3 * q + 1] += kSlab[s][q] * gn1;
                gN[3 * q + 2] += kSlab[s][q] * gn2;
            }
        }
        // N = M^-1:  dL/dM = -N^T dL/dN N^T; column b of M is a_b
        double T1[9];
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b)
                T1[3 * a + b] = N[a] * gN[b] + N[3 + a] * gN[3 + b] + N[6 + a] * gN[6 + b];
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b)
                ga[b][a] = -(T1[3 * a] * N[3 * b] + T1[3 * a + 1] * N[3 * b + 1] + T1[3 * a + 2] * N[3 * b + 2]);
    } else {
#pragma unroll
        for (int f = 0; f < 4; ++f) {
            const double gA = r[3 * f], gB = r[3 * f + 1], gDp = r[3 * f + 2];
            const int m0 = (f == 0) ? 1 : 0, m1 = (f <= 1) ? 2 : 1, m2 = (f <= 2) ? 3 : 2;
            const double* P0 = G.a[m0];
            const double e1[3] = {G.a[m1][0] - P0[0], G.a[m1][1] - P0[1], G.a[m1][2] - P0[2]};
            const double e2[3] = {G.a[m2][0] - P0[0], G.a[m2][1] - P0[1], G.a[m2][2] - P0[2]};
            double nv[3];
            cross3(e1, e2, nv);
            const double to_f = nv[0] * (G.a[f][0] - P0[0]) + nv[1] * (G.a[f][1] - P0[1]) + nv[2] * (G.a[f][2] - P0[2]);
            const double sgn = (to_f > 0.0) ? -1.0 : 1.0;
            for (int c = 0; c < 3; ++c) nv[c] *= sgn;
            const double nlen = sqrt(nv[0] * nv[0] + nv[1] * nv[1] + nv[2] * nv[2]);
            const double nz = clamp_nz(nv[2], nlen);
            const double A = -nv[0] / nz, B = -nv[1] / nz;
            // D' = P0z - A P0x - B P0y + A ox + B oy
            const double gAt = gA + gDp * (ox - P0[0]);
            const double gBt = gB + gDp * (oy - P0[1]);
            gox += gDp * A;
            goy += gDp * B;
            double gn[3] = {-gAt / nz * sgn, -gBt / nz * sgn, -(gAt * A + gBt * B) / nz * sgn};  // d(e1 x e2)
            double ge1[3], ge2[3];
            cross3(e2, gn, ge1);
            cross3(gn, e1, ge2);
            const double gP0[3] = {-gDp * A, -gDp * B, gDp};
            for (int c = 0; c < 3; ++c) {
                ga[m0][c] += gP0[c] - ge1[c] - ge2[c];
                ga[m1][c] += ge1[c];
                ga[m2][c] += ge2[c];
            }
        }
    }
    // ox = i0 + 1/2 - c_x, oy = j0 + 1/2 - c_y; c_z does not enter a chord
    const double gc0 = -gox, gc1 = -goy;
    // Sec. 3.4 "Adaptive Population Control": the view-space positional
    // gradient (dL/d centre x, y with the offsets fixed) per unit of
    // normalised device coordinates, and the screen radius
    {
        const double ex = gc0 * 0.5 * (double)V.width, ey = gc1 * 0.5 * (double)V.height;
        stat = make_float2((float)sqrt(ex * ex + ey * ey), (float)G.radius);
    }

    // ---- ray space -> camera: c = phi(t) with d phi/dt = J; a_k = J(t) oc_k
    const double* J = G.J;
    const double x = G.tc[0], y = G.tc[1], z = G.tc[2];
    const double l = G.c[2];
    double gt[3];
    for (int c = 0; c < 3; ++c) gt[c] = J[c] * gc0 + J[3 + c] * gc1;
    double gR[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    double gd[4] = {0, 0, 0, 0};
    const double iz2 = 1.0 / (z * z), il = 1.0 / l, il3 = il * il * il;
#pragma unroll
    for (int k = 0; k < ND; ++k) {
        double goc[3];
        for (int c = 0; c < 3; ++c) goc[c] = J[c] * ga[k][0] + J[3 + c] * ga[k][1] + J[6 + c] * ga[k][2];
        const double* w = G.oc[k];
        const double tw = x * w[0] + y * w[1] + z * w[2];
        // derivatives of J w with respect to t
        const double d00 = -V.fx * w[2] * iz2, d02 = -V.fx * w[0] * iz2 + 2.0 * V.fx * x * w[2] * iz2 / z;
        const double d11 = -V.fy * w[2] * iz2, d12 = -V.fy * w[1] * iz2 + 2.0 * V.fy * y * w[2] * iz2 / z;
        const double d20 = w[0] * il - tw * x * il3, d21 = w[1] * il - tw * y * il3, d22 = w[2] * il - tw * z * il3;
        gt[0] += d00 * ga[k][0] + d20 * ga[k][2];
        gt[1] += d11 * ga[k][1] + d21 * ga[k][2];
        gt[2] += d02 * ga[k][0] + d12 * ga[k][1] + d22 * ga[k][2];
        // camera -> world offset, then onto R and the distance
        double go[3];
        for (int c = 0; c < 3; ++c) go[c] = V.Rw[c] * goc[0] + V.Rw[3 + c] * goc[1] + V.Rw[6 + c] * goc[2];
        if (KIND == LINPRIM_OCTAHEDRON) {
            const double dk = (double)dv[k];
            for (int rr = 0; rr < 3; ++rr) {
                gR[3 * rr + k] += go[rr] * dk;
                gd[k] += go[rr] * G.R[3 * rr + k];
            }
        } else {
            const double gk = (double)dv[k] * kInvSqrt3;
            for (int rr = 0; rr < 3; ++rr) {
                const double rb = kTetDir[k][0] * G.R[3 * rr] + kTetDir[k][1] * G.R[3 * rr + 1] +
                                  kTetDir[k][2] * G.R[3 * rr + 2];
                for (int c = 0; c < 3; ++c) gR[3 * rr + c] += go[rr] * kTetDir[k][c] * gk;
                gd[k] += go[rr] * rb * kInvSqrt3;
            }
        }
    }
    double gm[3];
    for (int c = 0; c < 3; ++c) gm[c] = V.Rw[c] * gt[0] + V.Rw[3 + c] * gt[1] + V.Rw[6 + c] * gt[2];
    pack_slot_result(gm, gR, gd, r[16], r[17], r[18], r[19], res);
}

// Colour backward of one view (single precision): the colour gradient
// (zero where the raw colour was clamped) onto the SH coefficients (added to
// gsh, or stored to a row of dL/dSH by ShStore) and, through the viewing
// direction, onto the mean (added to gm).
template <int K, class S_>
__device__ inline void view_colour_bwd_t(S_& S, const float shp[48], const float mu[3], const ViewInfo& V, float er,
                                         float eg, float eb, double gm[3]) {
    float dir[3] = {(float)((double)mu[0] - V.cam_pos[0]), (float)((double)mu[1] - V.cam_pos[1]),
                    (float)((double)mu[2] - V.cam_pos[2])};
    const float dn = sqrtf(dir[0] * dir[0] + dir[1] * dir[1] + dir[2] * dir[2]);
    const float idn = 1.0f / dn;
    for (int q = 0; q < 3; ++q) dir[q] *= idn;
    float raw[3];
    sh_raw_f(K, shp, dir[0], dir[1], dir[2], raw);
    S.K = K;
    S.sh = shp;
    S.gr[0] = raw[0] > 0.0f ? er : 0.0f;
    S.gr[1] = raw[1] > 0.0f ? eg : 0.0f;
    S.gr[2] = raw[2] > 0.0f ? eb : 0.0f;
    S.gdir[0] = S.gdir[1] = S.gdir[2] = 0.0f;
    sh_backward(S, dir[0], dir[1], dir[2]);
    const float dot = S.gdir[0] * dir[0] + S.gdir[1] * dir[1] + S.gdir[2] * dir[2];
    for (int q = 0; q < 3; ++q) gm[q] += (double)((S.gdir[q] - dot * dir[q]) * idn);
}

template <int K>
__device__ inline void view_colour_bwd(const float shp[48], const float mu[3], const ViewInfo& V, float er, float eg,
                                       float eb, float gsh[48], double gm[3]) {
    ShBack S;
    S.gsh = gsh;
    view_colour_bwd_t<K>(S, shp, mu, V, er, eg, eb, gm);
}

// Rotation -> quaternion through R = I + s K(q), s = 2/|q|^2, and Eq. 1 ->
// opacity with min(d) held constant.
template <int KIND>
__device__ inline void rotation_opacity_bwd(const float qf[4], const float* dv, float alpha, const double gR[9],
                                            double gsig, double gq[4], double& ga) {
    constexpr int ND = (KIND == LINPRIM_OCTAHEDRON) ? 3 : 4;
    const double w = qf[0], qx = qf[1], qy = qf[2], qz = qf[3];
    const double n2 = w * w + qx * qx + qy * qy + qz * qz;
    for (int m = 0; m < 4; ++m) gq[m] = 0.0;
    if (n2 > 0.0) {
        const double s = 2.0 / n2;
        const double Km[9] = {-(qy * qy + qz * qz), qx * qy - w * qz, qx * qz + w * qy,
                              qx * qy + w * qz, -(qx * qx + qz * qz), qy * qz - w * qx,
                              qx * qz - w * qy, qy * qz + w * qx, -(qx * qx + qy * qy)};
        double gK = 0.0;
        for (int k = 0; k < 9; ++k) gK += gR[k] * Km[k];
        const double qv[4] = {w, qx, qy, qz};
        const double dK[4][9] = {{0, -qz, qy, qz, 0, -qx, -qy, qx, 0},
                                 {0, qy, qz, qy, -2 * qx, -w, qz, w, -2 * qx},
                                 {-2 * qy, qx, w, qx, 0, qz, -w, qz, -2 * qy},
                                 {-2 * qz, -w, qx, w, -2 * qz, qy, qx, qy, 0}};
#pragma unroll
        for (int mm = 0; mm < 4; ++mm) {
            double acc = -s * s * qv[mm] * gK;
            for (int k = 0; k < 9; ++k) acc += s * gR[k] * dK[mm][k];
            gq[mm] = acc;
        }
    }
    double dmin = (double)dv[0];
    for (int k = 1; k < ND; ++k) dmin = fmin(dmin, (double)dv[k]);
    const double al = (double)alpha;
    ga = gsig * kAlphaScaleD / ((1.0 - kAlphaScaleD * al) * 2.0 * dmin);
}

// ---------------------------------------------------------------------------
// Stage 1, the work of visible slot t: sums the slot's records, then the slot
// result (ray-space or exact variant).  With several views (DEG < 0) it is
// written back in place, into the slot's first record, for k_prim_bwd.  With
// one view (DEG >= 0) a primitive has at most one slot, so the thread
// finishes the primitive itself: colour -> SH and viewing direction, rotation
// -> quaternion, Eq. 1 -> opacity, and writes its gradients.
// ---------------------------------------------------------------------------
template <int KIND, bool EXACT, int DEG>
__device__ inline void slot_work(int64_t t, const float* __restrict__ means, const float* __restrict__ quats,
                                 const float* __restrict__ dists, const float* __restrict__ opacity,
                                 const float* __restrict__ sh, int64_t n, const ViewInfo* __restrict__ views,
                                 const float* __restrict__ payload, const uint32_t* __restrict__ tiles,
                                 const uint32_t* __restrict__ offsets, float* __restrict__ grads, int nq,
                                 const uint32_t* __restrict__ vis, int aa, float2* __restrict__ stats,
                                 float* __restrict__ g_means, float* __restrict__ g_quats, float* __restrict__ g_dists,
                                 float* __restrict__ g_opacity, float* __restrict__ g_sh) {
    const int64_t vs = vis[t];
    const int v = (int)(vs / n);
    const int64_t i = vs - (int64_t)v * n;
    constexpr int ND = (KIND == LINPRIM_OCTAHEDRON) ? 3 : 4;
    float4* rp = reinterpret_cast<float4*>(grads + (int64_t)offsets[vs] * nq * kGradWords);
    // the pixel rectangle: read here only where it decides which records
    // exist (several groups per tile); the plane origin below takes it from
    // the recomputed geometry, which reproduces the preprocessing's exactly
    const int4 rc = (nq == 1) ? make_int4(0, 0, 0, 0) : *reinterpret_cast<const int4*>(payload + vs * kRecordWords);
    const int nrec = (int)tiles[vs] * nq;
    // the primitive's inputs, loaded while the records are summed
    float mu[3], qv[4], dv[ND];
#pragma unroll
    for (int c = 0; c < 3; ++c) mu[c] = means[3 * i + c];
#pragma unroll
    for (int c = 0; c < 4; ++c) qv[c] = quats[4 * i + c];
#pragma unroll
    for (int c = 0; c < ND; ++c) dv[c] = dists[ND * i + c];
    const float alpha = opacity[i];
    float r[kGradWords];
#pragma unroll
    for (int k = 0; k < kGradWords; ++k) r[k] = 0.0f;
    if (nrec <= kMidRun) {
        // sum the run in record order (skipping groups the rectangle misses),
        // loading four records before adding them
        const int qx = (nq == 1) ? 1 : (nq == 4) ? 2 : 4, tile = 8 * qx;
        const int shift = (tile == 8) ? 3 : (tile == 16) ? 4 : 5;
        const int tx0 = rc.x >> shift, ty0 = rc.y >> shift, ntx = (rc.z >> shift) - tx0 + 1;
        for (int q0 = 0; q0 < nrec; q0 += 4) {
            float4 x[4][kGradWords / 4];
#pragma unroll
            for (int h = 0; h < 4; ++h) {
                const int q = q0 + h;
                const bool use = q < nrec && (nq == 1 || record_exists(q, nq, qx, tile, rc, tx0, ty0, ntx));
#pragma unroll
                for (int k = 0; k < kGradWords / 4; ++k)
                    x[h][k] = use ? rp[q * (kGradWords / 4) + k] : make_float4(0.f, 0.f, 0.f, 0.f);
            }
#pragma unroll
            for (int h = 0; h < 4; ++h)
#pragma unroll
                for (int k = 0; k < kGradWords / 4; ++k) {
                    r[4 * k] += x[h][k].x;
                    r[4 * k + 1] += x[h][k].y;
                    r[4 * k + 2] += x[h][k].z;
                    r[4 * k + 3] += x[h][k].w;
                }
        }
    } else {
        // the chunk sums k_sum_big left in each chunk's first record (one
        // chunk for a run of at most kBigRun records)
        const int nch = (nrec <= kBigRun) ? 1 : kBigChunks;
        for (int c = 0; c < nch; ++c) {
            const int q = big_chunk_start(c, nrec);
#pragma unroll
            for (int k = 0; k < kGradWords / 4; ++k) {
                const float4 x = rp[q * (kGradWords / 4) + k];
                r[4 * k] += x.x;
                r[4 * k + 1] += x.y;
                r[4 * k + 2] += x.z;
                r[4 * k + 3] += x.w;
            }
        }
    }
    const ViewInfo& V = views[v];
    Geom G;
    float res[kGradWords];
    if (build_geometry(KIND, EXACT, aa != 0, mu, qv, dv, alpha, V, G)) {
        // the plane origin of the record: the rectangle's centre (see k_preprocess)
        const double ox = 0.5 * (double)(G.rect[0] + G.rect[2]) + 0.5 - G.c[0];
        const double oy = 0.5 * (double)(G.rect[1] + G.rect[3]) + 0.5 - G.c[1];
        if (EXACT) {
            // the view-space positional gradient is a ray-space quantity: none here
            stats[vs] = make_float2(0.0f, (float)G.radius);
            double dmin = (double)dv[0];
            for (int k = 1; k < ND; ++k) dmin = fmin(dmin, (double)dv[k]);
            const double sigma = -log(1.0 - kAlphaScaleD * (double)alpha) / (2.0 * dmin);
            exact_slot_bwd<KIND>(G, V, dv, sigma, ox, oy, r, res);
        } else {
            float2 st;
            ray_slot_bwd<KIND>(G, V, dv, ox, oy, r, res, st);
            stats[vs] = st;
        }
    } else {
        // not reached for a slot the forward pass binned (same geometry)
        if (DEG < 0) return;
#pragma unroll
        for (int k = 0; k < kGradWords; ++k) res[k] = 0.0f;
    }
    // rotation -> quaternion and Eq. 1 -> opacity for this slot (linear in
    // the slot's dL/dR and dL/dsigma, so the per-view values sum to the
    // primitive's); the primitive's inputs are read again (cache hits) through
    // an index the compiler cannot see through, so that the first copies are
    // not held in registers across the geometry
    int64_t ii = i;
    asm volatile("" : "+v"(ii));
    float q2[4], d2[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) q2[c] = quats[4 * ii + c];
#pragma unroll
    for (int c = 0; c < ND; ++c) d2[c] = dists[ND * ii + c];
    const float al = opacity[ii];
    double gq[4], ga;
    {
        double gR[9];
        for (int c = 0; c < 9; ++c) gR[c] = res[3 + c];
        rotation_opacity_bwd<KIND>(q2, d2, al, gR, (double)res[19], gq, ga);
    }
    if (DEG < 0) {
        // the slot result, written back into the slot's first record:
        // [0..2] dL/d mu (geometric part), [3..6] dL/dq, [7..10] dL/d
        // distances, [11..13] dL/d rgb, [14] dL/d alpha
        rp[0] = make_float4(res[0], res[1], res[2], (float)gq[0]);
        rp[1] = make_float4((float)gq[1], (float)gq[2], (float)gq[3], res[12]);
        rp[2] = make_float4(res[13], res[14], res[15], res[16]);
        rp[3] = make_float4(res[17], res[18], (float)ga, 0.0f);
        return;
    }
    // one view: the primitive's gradients, written as they are formed
    constexpr int DG = (DEG < 0) ? 0 : DEG;
    constexpr int K = (DG + 1) * (DG + 1);
    for (int c = 0; c < 4; ++c) g_quats[4 * i + c] = (float)gq[c];
    for (int c = 0; c < ND; ++c) g_dists[ND * i + c] = res[12 + c];
    g_opacity[i] = (float)ga;
    float m2[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) m2[c] = means[3 * ii + c];
    float shp[48];
    load_sh<DG>(sh + i * (int64_t)K * 3, shp);
    double gm[3];
    for (int c = 0; c < 3; ++c) gm[c] = res[c];
    ShStore S;
    S.gs = g_sh + i * (int64_t)(3 * K);
    view_colour_bwd_t<K>(S, shp, m2, V, res[16], res[17], res[18], gm);
    for (int c = 0; c < 3; ++c) g_means[3 * i + c] = (float)gm[c];
}

// One view: zero gradients for the primitives without a slot (all of them
// when the pairs overflowed the capacity).  Thread t takes primitive t; the
// wave's SH rows, contiguous, are written together by all its lanes (four
// words per lane and store where a row is a whole number of float4s).
template <int KIND, int DEG>
__device__ inline void zero_unseen(const uint32_t* __restrict__ tiles, int64_t n, bool all, int64_t t,
                                   float* __restrict__ g_means, float* __restrict__ g_quats,
                                   float* __restrict__ g_dists, float* __restrict__ g_opacity,
                                   float* __restrict__ g_sh) {
    constexpr int ND = (KIND == LINPRIM_OCTAHEDRON) ? 3 : 4;
    constexpr int W = 3 * (DEG + 1) * (DEG + 1);
    constexpr int U = (W % 4 == 0) ? 4 : 1;   // words per store
    constexpr int UPR = W / U;                 // stores per primitive
    const int lane = threadIdx.x & 63;
    const bool unseen = t < n && (all || tiles[t] == 0);
    if (unseen) {
        for (int c = 0; c < 3; ++c) g_means[3 * t + c] = 0.0f;
        for (int c = 0; c < 4; ++c) g_quats[4 * t + c] = 0.0f;
        for (int c = 0; c < ND; ++c) g_dists[ND * t + c] = 0.0f;
        g_opacity[t] = 0.0f;
    }
    const uint64_t m = __ballot(unseen);
    if (m == 0) return;
    const int64_t u0 = (t - lane) * UPR;   // first store unit of the wave's rows
#pragma unroll 4
    for (int j = 0; j < UPR; ++j) {
        const int u = lane + 64 * j;
        if ((m >> (u / UPR)) & 1) {
            if (U == 4)
                reinterpret_cast<float4*>(g_sh)[u0 + u] = make_float4(0.f, 0.f, 0.f, 0.f);
            else
                g_sh[u0 + u] = 0.0f;
        }
    }
}

// Stage 1, one thread per (view, primitive) slot that touches a tile, taken
// from the list the scan built, so that no lane idles on a culled slot.  With
// one view the grid (one thread per primitive at least) also writes the zero
// gradients of the primitives without a slot, after the slot work (memory
// traffic that overlaps the arithmetic of the other waves).
template <int KIND, bool EXACT, int DEG>
__global__ __launch_bounds__(128, (DEG < 0 && KIND == LINPRIM_OCTAHEDRON) ? 3 : 1) void k_slot_bwd(const float* __restrict__ means, const float* __restrict__ quats,
                                                  const float* __restrict__ dists, const float* __restrict__ opacity,
                                                  const float* __restrict__ sh,
                                                  int64_t n, const ViewInfo* __restrict__ views,
                                                  const float* __restrict__ payload, const uint32_t* __restrict__ tiles,
                                                  const uint32_t* __restrict__ offsets, float* __restrict__ grads,
                                                  int nq, const Status* __restrict__ status, uint64_t capacity,
                                                  const uint32_t* __restrict__ vis, int aa,
                                                  float2* __restrict__ stats, float* __restrict__ g_means,
                                                  float* __restrict__ g_quats, float* __restrict__ g_dists,
                                                  float* __restrict__ g_opacity, float* __restrict__ g_sh) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool overflow = status->n_pairs > capacity;
    const int64_t n_vis = status->n_vis;
    if (DEG < 0) {
        if (!overflow && t < n_vis)
            slot_work<KIND, EXACT, DEG>(t, means, quats, dists, opacity, sh, n, views, payload, tiles, offsets, grads,
                                        nq, vis, aa, stats, g_means, g_quats, g_dists, g_opacity, g_sh);
        return;
    }
    // one view: the S blocks of slot work are spread evenly over the grid
    // (block b takes slot block b S / B when that is where the quotient steps),
    // so that slot arithmetic and zero stores run side by side
    const int64_t S = (n_vis + blockDim.x - 1) / blockDim.x, B = gridDim.x;
    const int64_t bs = (int64_t)blockIdx.x * S;
    if (!overflow && bs % B < S) {
        const int64_t ts = (bs / B) * blockDim.x + threadIdx.x;
        if (ts < n_vis)
            slot_work<KIND, EXACT, DEG>(ts, means, quats, dists, opacity, sh, n, views, payload, tiles, offsets, grads,
                                        nq, vis, aa, stats, g_means, g_quats, g_dists, g_opacity, g_sh);
    }
    zero_unseen<KIND, (DEG < 0 ? 0 : DEG)>(tiles, n, overflow, t, g_means, g_quats, g_dists, g_opacity, g_sh);
}

// ---------------------------------------------------------------------------
// Stage 2 (several views), one thread per primitive: sums the views' slot
// results (quaternion and opacity gradients already formed per slot) and
// runs the colour backward of each view.  Outputs are overwritten.
// ---------------------------------------------------------------------------
template <int KIND, int DEG>
__global__ __launch_bounds__(128) void k_prim_bwd(const float* __restrict__ means, const float* __restrict__ quats,
                                                  const float* __restrict__ dists, const float* __restrict__ opacity,
                                                  const float* __restrict__ sh, int64_t n, int n_views,
                                                  const ViewInfo* __restrict__ views,
                                                  const uint32_t* __restrict__ tiles,
                                                  const uint32_t* __restrict__ offsets, const float* __restrict__ grads,
                                                  int nq, const Status* __restrict__ status, uint64_t capacity,
                                                  float* __restrict__ g_means, float* __restrict__ g_quats,
                                                  float* __restrict__ g_dists, float* __restrict__ g_opacity,
                                                  float* __restrict__ g_sh) {
    // SH gradients summed over the views in LDS, coefficient-major with a
    // padded stride (word w of thread t at w * 129 + t), then stored coalesced
    constexpr int SP = 129;
    __shared__ float stage[48 * SP];
    const int64_t i0 = (int64_t)blockIdx.x * blockDim.x;
    const int64_t i = i0 + threadIdx.x;
    constexpr int ND = (KIND == LINPRIM_OCTAHEDRON) ? 3 : 4;
    constexpr int K = (DEG + 1) * (DEG + 1);
    const bool ok = status->n_pairs <= capacity && i < n;
    double gm[3] = {0, 0, 0}, gq[4] = {0, 0, 0, 0}, gd[4] = {0, 0, 0, 0}, ga = 0.0;
    float* acc = stage + threadIdx.x;
#pragma unroll
    for (int k = 0; k < 3 * K; ++k) acc[k * SP] = 0.0f;
    float shp[48], mu[3];
    bool seen = false;
    for (int v = 0; ok && v < n_views; ++v) {
        const int64_t vs = (int64_t)v * n + i;
        if (tiles[vs] == 0) continue;
        if (!seen) {
            load_sh<DEG>(sh + i * (int64_t)K * 3, shp);
            for (int c = 0; c < 3; ++c) mu[c] = means[3 * i + c];
            seen = true;
        }
        // the slot result k_slot_bwd left in the slot's first record
        const float4* rp = reinterpret_cast<const float4*>(grads + (int64_t)offsets[vs] * nq * kGradWords);
        const float4 a = rp[0], b = rp[1], c = rp[2], d = rp[3];
        gm[0] += a.x; gm[1] += a.y; gm[2] += a.z;
        gq[0] += a.w; gq[1] += b.x; gq[2] += b.y; gq[3] += b.z;
        gd[0] += b.w; gd[1] += c.x; gd[2] += c.y; gd[3] += c.z;
        ga += d.z;
        ShLds S;
        S.acc = acc;
        S.stride = SP;
        view_colour_bwd_t<K>(S, shp, mu, views[v], c.w, d.x, d.y, gm);
    }
    if (i < n) {
        for (int c = 0; c < 3; ++c) g_means[3 * i + c] = (float)gm[c];
        for (int c = 0; c < 4; ++c) g_quats[4 * i + c] = (float)gq[c];
        for (int c = 0; c < ND; ++c) g_dists[ND * i + c] = (float)gd[c];
        g_opacity[i] = (float)ga;
    }
    // the block's [128][3K] slab of SH gradients, stored coalesced
    const int w3 = 3 * K;
    __syncthreads();
    const int64_t rows = (n - i0) < 128 ? (n - i0) : 128;
    float* gs = g_sh + i0 * (int64_t)w3;
    for (int64_t j = threadIdx.x; j < rows * w3; j += 128) {
        const int64_t r = j / w3;
        gs[j] = stage[(j - r * w3) * SP + r];
    }
}

hipError_t launch_preprocess_bwd(const linprim_prims& p, int32_t n_views, int tile, bool exact, bool aa,
                                 const ViewLayout& L,
                                 const char* vws, const PairLayout& P, const char* pws, float* g_means,
                                 float* g_quats, float* g_dists, float* g_opacity, float* g_sh, hipStream_t stream) {
    if (p.n == 0) return hipSuccess;
    const ViewInfo* views = reinterpret_cast<const ViewInfo*>(vws + L.views);
    const float* payload = reinterpret_cast<const float*>(vws + L.payload);
    const uint32_t* tiles = reinterpret_cast<const uint32_t*>(vws + L.tiles);
    const uint32_t* offsets = reinterpret_cast<const uint32_t*>(vws + L.offsets);
    const Status* st = reinterpret_cast<const Status*>(vws + L.status);
    float* grads = reinterpret_cast<float*>(const_cast<char*>(pws) + P.grads);
    const int nq = (tile / 8) * (tile / 8);
    const uint64_t cap = (uint64_t)P.capacity;
    const int64_t vn = p.n * (int64_t)n_views;
    const uint32_t* big = reinterpret_cast<const uint32_t*>(vws + L.big);
    // a fixed grid of waves strides over the (big slot, chunk) items, whose
    // number is only known on the device
    const int64_t max_waves = (vn * kBigChunks + 3) / 4;   // bounds the grid only
    const unsigned big_blocks = (unsigned)(max_waves < 1024 ? (max_waves > 0 ? max_waves : 1) : 1024);
    const uint32_t* huge = reinterpret_cast<const uint32_t*>(vws + L.huge);
    hipLaunchKernelGGL(k_sum_big, dim3(big_blocks), dim3(256), 0, stream, payload, tiles, offsets, big, huge, vn, tile,
                       st, cap, grads);
    const dim3 g1((unsigned)((vn + 127) / 128));
    const uint32_t* vis = reinterpret_cast<const uint32_t*>(vws + L.vis);
    float2* stats = reinterpret_cast<float2*>(const_cast<char*>(vws) + L.stats);
    const dim3 g2((unsigned)((p.n + 127) / 128));
    const bool one = n_views == 1;
#define LP_SLOT(K_, E_, D_)                                                                                     \
    hipLaunchKernelGGL((k_slot_bwd<K_, E_, D_>), g1, dim3(128), 0, stream, p.means, p.quats, p.dists, p.opacity, \
                       p.sh, p.n, views, payload, tiles, offsets, grads, nq, st, cap, vis, aa ? 1 : 0, stats,   \
                       g_means, g_quats, g_dists, g_opacity, g_sh)
#define LP_STAGES(K_, E_, D_)                                                                                     \
    if (one) {                                                                                                     \
        LP_SLOT(K_, E_, D_);                                                                                       \
    } else {                                                                                                       \
        LP_SLOT(K_, E_, -1);                                                                                       \
        hipLaunchKernelGGL((k_prim_bwd<K_, D_>), g2, dim3(128), 0, stream, p.means, p.quats, p.dists, p.opacity,  \
                           p.sh, p.n, n_views, views, tiles, offsets, grads, nq, st, cap, g_means, g_quats,       \
                           g_dists, g_opacity, g_sh);                                                              \
    }
#define LP_DEG(K_, E_)                          \
    switch (p.sh_degree) {                      \
        case 0: LP_STAGES(K_, E_, 0) break;     \
        case 1: LP_STAGES(K_, E_, 1) break;     \
        case 2: LP_STAGES(K_, E_, 2) break;     \
        default: LP_STAGES(K_, E_, 3) break;    \
    }
    if (p.type == LINPRIM_OCTAHEDRON) {
        if (exact) LP_DEG(LINPRIM_OCTAHEDRON, true) else LP_DEG(LINPRIM_OCTAHEDRON, false)
    } else {
        if (exact) LP_DEG(LINPRIM_TETRAHEDRON, true) else LP_DEG(LINPRIM_TETRAHEDRON, false)
    }
#undef LP_DEG
#undef LP_STAGES
#undef LP_SLOT
    return hipGetLastError();
}

}  // namespace linprim
