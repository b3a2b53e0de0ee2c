// k_population.hip -- adaptive population control (Sec. 3.4 "Adaptive
// Population Control"; thresholds in App. G): statistics accumulated over
// the views of each step, then one densify / prune pass that compacts the
// primitives and their Adam moments into new arrays.
//
//   k_accum_stats   per primitive: add, over the views in which it touches a
//                   tile, the norm of its view-space positional gradient
//                   (left per slot by the preprocessing backward), count the
//                   views, keep the largest screen radius.
//   k_dens_count    per primitive: how many rows it leaves (0..3); block sums.
//   k_dens_scan     exclusive scan of the block sums (one block).
//   k_dens_apply    per primitive: its rows' offset (block scan) and the rows:
//                   the original or its two split children, then its clone.
#include <mutex>

#include "linprim_common.h"

namespace linprim {

__global__ __launch_bounds__(256) void k_accum_stats(int64_t n, int n_views, const uint32_t* __restrict__ tiles,
                                                     const float2* __restrict__ stats, float* __restrict__ grad_accum,
                                                     int32_t* __restrict__ count, float* __restrict__ max_radius) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float acc = 0.0f, mr = max_radius[i];
    int cnt = 0;
    for (int v = 0; v < n_views; ++v) {
        const int64_t vs = (int64_t)v * n + i;
        if (tiles[vs] == 0) continue;
        const float2 s = stats[vs];
        acc += s.x;
        mr = fmaxf(mr, s.y);
        ++cnt;
    }
    grad_accum[i] += acc;
    count[i] += cnt;
    max_radius[i] = mr;
}

hipError_t launch_accumulate_stats(int64_t n, int32_t n_views, const ViewLayout& L, const char* vws,
                                   float* grad_accum, int32_t* count, float* max_radius, hipStream_t s) {
    if (n == 0) return hipSuccess;
    const uint32_t* tiles = reinterpret_cast<const uint32_t*>(vws + L.tiles);
    const float2* stats = reinterpret_cast<const float2*>(vws + L.stats);
    hipLaunchKernelGGL(k_accum_stats, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, (int)n_views, tiles,
                       stats, grad_accum, count, max_radius);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Decisions, in float32 (the precision of every input): size = longest axis
// 2 max d (octahedron) or sqrt(2) times the distance to the furthest corner
// (tetrahedron); a mean gradient above the threshold makes a candidate, a
// small candidate is cloned, a larger one split in two; transparent, too
// large or (originals only) too wide primitives are removed.
// ---------------------------------------------------------------------------
struct Decision {
    bool keep, split, clone;
    __device__ int rows() const { return (keep ? 1 : 0) + (split ? 2 : 0) + (clone ? 1 : 0); }
};

template <int ND>
__device__ inline Decision decide(int type, const float* __restrict__ d, float opacity, float acc, int cnt,
                                  float mr, const DensifyParams& dp, float extent) {
    float dm = d[0];
#pragma unroll
    for (int k = 1; k < ND; ++k) dm = fmaxf(dm, d[k]);
    const float size = (type == LINPRIM_OCTAHEDRON) ? 2.0f * dm : (float)1.41421356237309504880 * dm;
    const float avg = cnt > 0 ? acc / (float)cnt : 0.0f;
    const float max_size = dp.max_size_frac * extent;
    const bool cand = avg > dp.grad_threshold;
    const bool small = size < dp.clone_size_frac * extent;
    const bool transparent = opacity < dp.min_opacity;
    Decision D;
    const bool split = cand && !small;
    D.keep = !split && !transparent && !(size > max_size) && !(mr > dp.max_radius);
    D.split = split && !transparent && !(size / dp.shrink > max_size);
    D.clone = cand && small && !transparent && !(size > max_size);
    return D;
}

template <int ND>
__global__ __launch_bounds__(256) void k_dens_count(int type, int64_t n, const float* __restrict__ dists,
                                                    const float* __restrict__ opacity,
                                                    const float* __restrict__ grad_accum,
                                                    const int32_t* __restrict__ count,
                                                    const float* __restrict__ max_radius, DensifyParams dp,
                                                    float extent, int64_t* __restrict__ block_sums) {
    __shared__ int64_t part[256];
    const int t = threadIdx.x;
    int64_t sum = 0;
#pragma unroll
    for (int k = 0; k < kDensifyItems / 256; ++k) {
        const int64_t i = (int64_t)blockIdx.x * kDensifyItems + k * 256 + t;
        if (i < n) sum += decide<ND>(type, dists + ND * i, opacity[i], grad_accum[i], count[i], max_radius[i], dp,
                                     extent).rows();
    }
    part[t] = sum;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (t < off) part[t] += part[t + off];
        __syncthreads();
    }
    if (t == 0) block_sums[blockIdx.x] = part[0];
}

// Exclusive scan of nb block sums in place; block_sums[nb] = total.
__global__ __launch_bounds__(1024) void k_dens_scan(int64_t* __restrict__ block_sums, int64_t nb) {
    __shared__ int64_t s[1024];
    __shared__ int64_t carry;
    const int t = threadIdx.x;
    if (t == 0) carry = 0;
    __syncthreads();
    for (int64_t base = 0; base < nb; base += 1024) {
        const int64_t i = base + t;
        const int64_t x = i < nb ? block_sums[i] : 0;
        s[t] = x;
        __syncthreads();
        for (int off = 1; off < 1024; off <<= 1) {
            const int64_t y = t >= off ? s[t - off] : 0;
            __syncthreads();
            s[t] += y;
            __syncthreads();
        }
        if (i < nb) block_sums[i] = carry + s[t] - x;
        __syncthreads();
        if (t == 1023) carry += s[1023];
        __syncthreads();
    }
    if (t == 0) block_sums[nb] = carry;
}

// One output row of every field of the state: a copy of source row i, with
// its Adam moments (kept primitives) or zero moments (new primitives).
__device__ inline void copy_row(const StateSet& src, const StateSet& dst, const int width[5], int64_t i, int64_t o,
                                bool keep_moments) {
#pragma unroll
    for (int f = 0; f < 5; ++f) {
        const int w = width[f];
        const float* sp = src.p[f] + i * w;
        float* dp = dst.p[f] + o * w;
        for (int k = 0; k < w; ++k) dp[k] = sp[k];
        if (dst.m[f]) {
            float* dm = dst.m[f] + o * w;
            float* dv = dst.v[f] + o * w;
            if (keep_moments && src.m[f]) {
                const float* sm = src.m[f] + i * w;
                const float* sv = src.v[f] + i * w;
                for (int k = 0; k < w; ++k) {
                    dm[k] = sm[k];
                    dv[k] = sv[k];
                }
            } else {
                for (int k = 0; k < w; ++k) {
                    dm[k] = 0.0f;
                    dv[k] = 0.0f;
                }
            }
        }
    }
}

template <int ND>
__global__ __launch_bounds__(256) void k_dens_apply(int type, int64_t n, StateSet src, StateSet dst, int sh_floats,
                                                    const float* __restrict__ normals,
                                                    const float* __restrict__ grad_accum,
                                                    const int32_t* __restrict__ count,
                                                    const float* __restrict__ max_radius, DensifyParams dp,
                                                    float extent, const int64_t* __restrict__ block_sums) {
    constexpr int PER = kDensifyItems / 256;
    __shared__ int64_t s[256];
    const int t = threadIdx.x;
    // this thread's items are consecutive, so that the block's rows stay in order
    const int64_t i0 = (int64_t)blockIdx.x * kDensifyItems + (int64_t)t * PER;
    Decision D[PER];
    int64_t mine = 0;
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        const int64_t i = i0 + k;
        D[k] = (i < n) ? decide<ND>(type, src.p[2] + ND * i, src.p[3][i], grad_accum[i], count[i], max_radius[i], dp,
                                    extent)
                       : Decision{false, false, false};
        mine += D[k].rows();
    }
    s[t] = mine;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
        const int64_t y = t >= off ? s[t - off] : 0;
        __syncthreads();
        s[t] += y;
        __syncthreads();
    }
    int64_t o = block_sums[blockIdx.x] + s[t] - mine;
    const int width[5] = {3, 4, ND, 1, sh_floats};
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        const int64_t i = i0 + k;
        if (i >= n) break;
        if (D[k].keep) copy_row(src, dst, width, i, o++, true);
        if (D[k].split) {
            // children: distances / shrink; positions mu + R (d * z) along the
            // octahedron's own axes, or mu + (max d / 2) z for a tetrahedron
            const float* d = src.p[2] + ND * i;
            const float* q = src.p[1] + 4 * i;
            double R[9];
            const bool rot = quat_rotation_d((double)q[0], (double)q[1], (double)q[2], (double)q[3], R);
            float dm = d[0];
#pragma unroll
            for (int kk = 1; kk < ND; ++kk) dm = fmaxf(dm, d[kk]);
            for (int c = 0; c < 2; ++c) {
                copy_row(src, dst, width, i, o, false);
                const float* z = normals + (i * 2 + c) * 3;
                double off[3];
                if (type == LINPRIM_OCTAHEDRON) {
                    const double l[3] = {(double)d[0] * z[0], (double)d[1] * z[1], (double)d[2] * z[2]};
                    for (int r = 0; r < 3; ++r)
                        off[r] = rot ? R[3 * r] * l[0] + R[3 * r + 1] * l[1] + R[3 * r + 2] * l[2] : l[r];
                } else {
                    for (int r = 0; r < 3; ++r) off[r] = 0.5 * (double)dm * (double)z[r];
                }
                float* mu = dst.p[0] + o * 3;
                const float* mus = src.p[0] + i * 3;
                for (int r = 0; r < 3; ++r) mu[r] = (float)((double)mus[r] + off[r]);
                float* dd = dst.p[2] + o * ND;
                for (int kk = 0; kk < ND; ++kk) dd[kk] = (float)((double)d[kk] / (double)dp.shrink);
                ++o;
            }
        }
        if (D[k].clone) copy_row(src, dst, width, i, o++, false);
    }
}

hipError_t launch_densify_plan(int type, int64_t n, const float* dists, const float* opacity,
                               const float* grad_accum, const int32_t* count, const float* max_radius,
                               const DensifyParams& dp, float extent, int64_t* block_sums, hipStream_t s) {
    const int64_t nb = (n + kDensifyItems - 1) / kDensifyItems;
    if (nb > 0) {
        if (type == LINPRIM_OCTAHEDRON)
            hipLaunchKernelGGL(k_dens_count<3>, dim3((unsigned)nb), dim3(256), 0, s, type, n, dists, opacity,
                               grad_accum, count, max_radius, dp, extent, block_sums);
        else
            hipLaunchKernelGGL(k_dens_count<4>, dim3((unsigned)nb), dim3(256), 0, s, type, n, dists, opacity,
                               grad_accum, count, max_radius, dp, extent, block_sums);
    }
    hipLaunchKernelGGL(k_dens_scan, dim3(1), dim3(1024), 0, s, block_sums, nb);
    return hipGetLastError();
}

hipError_t launch_densify_apply(int type, int sh_degree, int64_t n, const StateSet& src, const float* normals,
                                const float* grad_accum, const int32_t* count, const float* max_radius,
                                const DensifyParams& dp, float extent, const int64_t* block_sums,
                                const StateSet& dst, hipStream_t s) {
    const int64_t nb = (n + kDensifyItems - 1) / kDensifyItems;
    if (nb == 0) return hipSuccess;
    const int shf = 3 * (sh_degree + 1) * (sh_degree + 1);
    if (type == LINPRIM_OCTAHEDRON)
        hipLaunchKernelGGL(k_dens_apply<3>, dim3((unsigned)nb), dim3(256), 0, s, type, n, src, dst, shf, normals,
                           grad_accum, count, max_radius, dp, extent, block_sums);
    else
        hipLaunchKernelGGL(k_dens_apply<4>, dim3((unsigned)nb), dim3(256), 0, s, type, n, src, dst, shf, normals,
                           grad_accum, count, max_radius, dp, extent, block_sums);
    return hipGetLastError();
}

// Scratch of the allocation-free densify entry point: the plan's block sums
// and total, (n / kDensifyItems + 1) values, held by each device the
// library runs on until the process ends.  Host code reaches it only through
// the address hipGetSymbolAddress returns for the current device.
constexpr int64_t kDensifyScratchItems = kNoAllocMaxPrims / kDensifyItems + 8;
static __device__ __align__(256) int64_t scratch[kDensifyScratchItems];

namespace {
constexpr int kScratchDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kScratchDevices];
}  // namespace

hipError_t densify_scratch(int64_t** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kScratchDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[dev] = p;
    }
    *out = static_cast<int64_t*>(g_scratch_ptr[dev]);
    return hipSuccess;
}

}  // namespace linprim
