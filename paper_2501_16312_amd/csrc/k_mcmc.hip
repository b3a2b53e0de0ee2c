// k_mcmc.hip -- LinPrim-MCMC's population steps (Sec. 3.4 "LinPrim-MCMC":
// GS-MCMC's relocation and noise applied to octahedra treated as Gaussians
// with standard deviations d / 2.6).
//
// Relocation, with caller-supplied 32-bit random numbers:
//   k_mc_count    per block of 1,024: sums of the integer weights
//                 w_i = floor(alpha_i 2^32) of live primitives (alpha > 0.005)
//                 and of the dead flags;
//   k_mc_scan     exclusive scan of both block sums (one block);
//   k_mc_prefix   inclusive weight prefix per primitive, list of the dead;
//   k_mc_sample   the k-th dead primitive draws a source: the first index whose
//                 prefix exceeds floor(total r_k / 2^32) (binary search);
//                 per-source draw counts by integer atomics;
//   k_mc_sources  a source drawn c times becomes one of N = min(c + 1, 51)
//                 copies: opacity 1 - (1 - alpha)^(1/N), distances scaled to
//                 keep the composited opacity's line integral; moments reset;
//   k_mc_copy     dead primitive k <- its (updated) source; moments reset.
// Noise: k_mc_noise adds noise_lr lr s(1 - alpha) R S^2 R^T eps to the centre.
// All decisions on integers; the sampling is exact and reproducible.
#include "linprim_common.h"

namespace linprim {

constexpr float kMcDead = 0.005f;
constexpr int kMcItems = 1024;
constexpr int kMcMaxN = 51;

__device__ inline uint64_t mc_weight(float a) {
    return a > kMcDead ? (uint64_t)floor((double)a * 4294967296.0) : 0ull;
}

__global__ __launch_bounds__(256) void k_mc_count(int64_t n, const float* __restrict__ opacity,
                                                  uint64_t* __restrict__ wsum, int64_t* __restrict__ dsum) {
    __shared__ uint64_t sw[256];
    __shared__ int64_t sd[256];
    const int t = threadIdx.x;
    uint64_t w = 0;
    int64_t d = 0;
#pragma unroll
    for (int k = 0; k < kMcItems / 256; ++k) {
        const int64_t i = (int64_t)blockIdx.x * kMcItems + (int64_t)t * (kMcItems / 256) + k;
        if (i < n) {
            const float a = opacity[i];
            w += mc_weight(a);
            d += a <= kMcDead ? 1 : 0;
        }
    }
    sw[t] = w;
    sd[t] = d;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (t < off) {
            sw[t] += sw[t + off];
            sd[t] += sd[t + off];
        }
        __syncthreads();
    }
    if (t == 0) {
        wsum[blockIdx.x] = sw[0];
        dsum[blockIdx.x] = sd[0];
    }
}

// Exclusive scans of nb block sums in place; entry nb receives the total.
__global__ __launch_bounds__(1024) void k_mc_scan(uint64_t* __restrict__ wsum, int64_t* __restrict__ dsum,
                                                  int64_t nb) {
    __shared__ uint64_t sw[1024];
    __shared__ int64_t sd[1024];
    __shared__ uint64_t cw;
    __shared__ int64_t cd;
    const int t = threadIdx.x;
    if (t == 0) {
        cw = 0;
        cd = 0;
    }
    __syncthreads();
    for (int64_t base = 0; base < nb; base += 1024) {
        const int64_t i = base + t;
        const uint64_t xw = i < nb ? wsum[i] : 0;
        const int64_t xd = i < nb ? dsum[i] : 0;
        sw[t] = xw;
        sd[t] = xd;
        __syncthreads();
        for (int off = 1; off < 1024; off <<= 1) {
            const uint64_t yw = t >= off ? sw[t - off] : 0;
            const int64_t yd = t >= off ? sd[t - off] : 0;
            __syncthreads();
            sw[t] += yw;
            sd[t] += yd;
            __syncthreads();
        }
        if (i < nb) {
            wsum[i] = cw + sw[t] - xw;
            dsum[i] = cd + sd[t] - xd;
        }
        __syncthreads();
        if (t == 1023) {
            cw += sw[1023];
            cd += sd[1023];
        }
        __syncthreads();
    }
    if (t == 0) {
        wsum[nb] = cw;
        dsum[nb] = cd;
    }
}

__global__ __launch_bounds__(256) void k_mc_prefix(int64_t n, const float* __restrict__ opacity,
                                                   const uint64_t* __restrict__ wsum,
                                                   const int64_t* __restrict__ dsum, uint64_t* __restrict__ prefix,
                                                   int32_t* __restrict__ dead_list, int32_t* __restrict__ counts) {
    constexpr int PER = kMcItems / 256;
    __shared__ uint64_t sw[256];
    __shared__ int64_t sd[256];
    const int t = threadIdx.x;
    const int64_t i0 = (int64_t)blockIdx.x * kMcItems + (int64_t)t * PER;
    uint64_t w[PER];
    bool dead[PER];
    uint64_t mw = 0;
    int64_t md = 0;
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        const int64_t i = i0 + k;
        const float a = i < n ? opacity[i] : 1.0f;
        w[k] = i < n ? mc_weight(a) : 0ull;
        dead[k] = i < n && a <= kMcDead;
        mw += w[k];
        md += dead[k] ? 1 : 0;
    }
    sw[t] = mw;
    sd[t] = md;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
        const uint64_t yw = t >= off ? sw[t - off] : 0;
        const int64_t yd = t >= off ? sd[t - off] : 0;
        __syncthreads();
        sw[t] += yw;
        sd[t] += yd;
        __syncthreads();
    }
    uint64_t run = wsum[blockIdx.x] + sw[t] - mw;
    int64_t rank = dsum[blockIdx.x] + sd[t] - md;
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        const int64_t i = i0 + k;
        if (i >= n) break;
        run += w[k];
        prefix[i] = run;
        counts[i] = 0;
        if (dead[k]) dead_list[rank++] = (int32_t)i;
    }
}

// n_draws >= 0: that many draws (adding primitives); otherwise one per dead
// primitive (the device count).
__global__ __launch_bounds__(256) void k_mc_sample(int64_t n, const uint64_t* __restrict__ prefix,
                                                   const uint64_t* __restrict__ wtotal,
                                                   const int64_t* __restrict__ dtotal, int64_t n_draws,
                                                   const uint32_t* __restrict__ rnd, int32_t* __restrict__ samples,
                                                   int32_t* __restrict__ counts) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t total = *wtotal;
    if (k >= (n_draws >= 0 ? n_draws : *dtotal) || total == 0) return;
    // floor(total r / 2^32), exactly
    const uint64_t r = rnd[k];
    const uint64_t t = (total >> 32) * r + (((total & 0xffffffffull) * r) >> 32);
    int64_t lo = 0, hi = n - 1;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (prefix[mid] > t) hi = mid; else lo = mid + 1;
    }
    samples[k] = (int32_t)lo;
    atomicAdd(counts + lo, 1);
}

__device__ inline void zero_moments(const StateSet& S, const int width[5], int64_t i) {
    if (!S.m[0]) return;
#pragma unroll
    for (int f = 0; f < 5; ++f)
        for (int k = 0; k < width[f]; ++k) {
            S.m[f][i * width[f] + k] = 0.0f;
            S.v[f][i * width[f] + k] = 0.0f;
        }
}

__global__ __launch_bounds__(256) void k_mc_sources(int64_t n, StateSet S, int sh_floats,
                                                    const int32_t* __restrict__ counts) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || counts[i] == 0) return;
    const int N = min(counts[i] + 1, kMcMaxN);
    const double a = (double)S.p[3][i];
    double an = 1.0 - pow(1.0 - a, 1.0 / (double)N);
    an = fmin(fmax(an, (double)kMcDead), 1.0 - 1.1920928955078125e-7);
    // sum_{j=1}^{N} sum_{k=0}^{j-1} C(j-1, k) (-1)^k an^(k+1) / sqrt(k+1)
    double denom = 0.0;
    for (int j = 1; j <= N; ++j) {
        double c = 1.0;                       // C(j-1, k)
        double p = an;                        // an^(k+1)
        for (int k = 0; k < j; ++k) {
            denom += ((k & 1) ? -c : c) * p / sqrt((double)(k + 1));
            c = c * (double)(j - 1 - k) / (double)(k + 1);
            p *= an;
        }
    }
    const double coeff = a / denom;
#pragma unroll
    for (int k = 0; k < 3; ++k) S.p[2][i * 3 + k] = (float)((double)S.p[2][i * 3 + k] * coeff);
    S.p[3][i] = (float)an;
    const int width[5] = {3, 4, 3, 1, sh_floats};
    zero_moments(S, width, i);
}

// Draw k's target: the k-th dead primitive, or row append_base + k when
// adding (n_draws >= 0).
__global__ __launch_bounds__(256) void k_mc_copy(StateSet S, int sh_floats, const int64_t* __restrict__ dtotal,
                                                 int64_t n_draws, int64_t append_base,
                                                 const uint64_t* __restrict__ wtotal,
                                                 const int32_t* __restrict__ dead_list,
                                                 const int32_t* __restrict__ samples) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= (n_draws >= 0 ? n_draws : *dtotal) || *wtotal == 0) return;
    const int64_t j = n_draws >= 0 ? append_base + k : (int64_t)dead_list[k], s = samples[k];
    const int width[5] = {3, 4, 3, 1, sh_floats};
#pragma unroll
    for (int f = 0; f < 5; ++f)
        for (int q = 0; q < width[f]; ++q) S.p[f][j * width[f] + q] = S.p[f][s * width[f] + q];
    zero_moments(S, width, j);
}

__global__ __launch_bounds__(256) void k_mc_noise(int64_t n, float* __restrict__ means,
                                                  const float* __restrict__ quats, const float* __restrict__ dists,
                                                  const float* __restrict__ opacity, const float* __restrict__ eps,
                                                  double scale) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double a = (double)opacity[i];
    const double gate = 1.0 / (1.0 + exp(-100.0 * ((1.0 - a) - 0.995)));
    double R[9];
    if (!quat_rotation_d((double)quats[4 * i], (double)quats[4 * i + 1], (double)quats[4 * i + 2],
                         (double)quats[4 * i + 3], R))
        return;
    double l[3];
    // R S^2 R^T e: into the primitive's frame, scale by (d / 2.6)^2, back
    for (int c = 0; c < 3; ++c) {
        const double e = R[c] * eps[3 * i] + R[3 + c] * eps[3 * i + 1] + R[6 + c] * eps[3 * i + 2];
        const double s = (double)dists[3 * i + c] / 2.6;
        l[c] = s * s * e;
    }
    for (int r = 0; r < 3; ++r)
        means[3 * i + r] = (float)((double)means[3 * i + r] + scale * gate * (R[3 * r] * l[0] + R[3 * r + 1] * l[1] +
                                                                             R[3 * r + 2] * l[2]));
}

// Workspace: prefix [n] u64 | wsum [nb+1] u64 | dsum [nb+1] i64 | dead [n] i32 | samples [n] i32 | counts [n] i32
// (draws when adding are at most n: the workspace of n serves both steps).
struct McLayout {
    size_t prefix, wsum, dsum, dead, samples, counts, total;
};

McLayout mc_layout(int64_t n) {
    const int64_t nb = (n + kMcItems - 1) / kMcItems;
    McLayout L;
    size_t off = 0;
    L.prefix = off; off = align256(off + (size_t)n * 8);
    L.wsum = off; off = align256(off + (size_t)(nb + 1) * 8);
    L.dsum = off; off = align256(off + (size_t)(nb + 1) * 8);
    L.dead = off; off = align256(off + (size_t)n * 4);
    L.samples = off; off = align256(off + (size_t)n * 4);
    L.counts = off; off = align256(off + (size_t)n * 4);
    L.total = off;
    return L;
}

size_t mc_workspace_bytes(int64_t n) { return mc_layout(n).total; }

// n_add < 0: relocate the dead in place; n_add >= 0: draw n_add sources
// among the first n rows and write their copies to rows n .. n + n_add - 1.
hipError_t launch_mc_relocate(int64_t n, int64_t n_add, int sh_degree, const StateSet& S, const uint32_t* rnd,
                              char* ws, hipStream_t s) {
    if (n == 0 || n_add == 0) return hipSuccess;
    const McLayout L = mc_layout(n);
    const int64_t nb = (n + kMcItems - 1) / kMcItems;
    uint64_t* prefix = (uint64_t*)(ws + L.prefix);
    uint64_t* wsum = (uint64_t*)(ws + L.wsum);
    int64_t* dsum = (int64_t*)(ws + L.dsum);
    int32_t* dead = (int32_t*)(ws + L.dead);
    int32_t* samples = (int32_t*)(ws + L.samples);
    int32_t* counts = (int32_t*)(ws + L.counts);
    const int shf = 3 * (sh_degree + 1) * (sh_degree + 1);
    const unsigned g1 = (unsigned)((n + 255) / 256);
    hipLaunchKernelGGL(k_mc_count, dim3((unsigned)nb), dim3(256), 0, s, n, S.p[3], wsum, dsum);
    hipLaunchKernelGGL(k_mc_scan, dim3(1), dim3(1024), 0, s, wsum, dsum, nb);
    hipLaunchKernelGGL(k_mc_prefix, dim3((unsigned)nb), dim3(256), 0, s, n, S.p[3], wsum, dsum, prefix, dead, counts);
    const int64_t draws_max = n_add >= 0 ? n_add : n;
    const unsigned gd = (unsigned)((draws_max + 255) / 256);
    hipLaunchKernelGGL(k_mc_sample, dim3(gd), dim3(256), 0, s, n, prefix, wsum + nb, dsum + nb, n_add, rnd, samples,
                       counts);
    hipLaunchKernelGGL(k_mc_sources, dim3(g1), dim3(256), 0, s, n, S, shf, counts);
    hipLaunchKernelGGL(k_mc_copy, dim3(gd), dim3(256), 0, s, S, shf, dsum + nb, n_add, n, wsum + nb, dead, samples);
    return hipGetLastError();
}

hipError_t launch_mc_noise(int64_t n, float* means, const float* quats, const float* dists, const float* opacity,
                           const float* eps, double scale, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_mc_noise, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, means, quats, dists, opacity,
                       eps, scale);
    return hipGetLastError();
}

int64_t mc_dead_offset(int64_t n) {
    const McLayout L = mc_layout(n);
    return (int64_t)(L.dsum + ((n + kMcItems - 1) / kMcItems) * 8);
}

}  // namespace linprim
