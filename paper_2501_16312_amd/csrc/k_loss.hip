// k_loss.hip -- the photometric loss of the optimisation (Sec. 3.4
// "Optimization": 3DGS's L1 + SSIM) and its gradient with respect to the
// rendered image, fused: per view and channel,
//   L = (1 - lam) mean |x - y| + lam (1 - mean s),
//   s = (2 mx my + C1)(2 sxy + C2) / ((mx^2 + my^2 + C1)(sxx + syy + C2)),
// local statistics by an 11 x 11 Gaussian window (sigma 1.5, zero padding).
//
// Two passes over 32 x 32 output tiles, each staging a 42 x 42 input tile
// (5-pixel halo) in LDS and applying the separable window as a row pass then
// a column pass:
//   k_ssim_fwd  five statistics -> s and its partial derivatives with respect
//               to mx, E[x^2], E[xy] (written per pixel), block sums of s and
//               |x - y|;
//   k_ssim_bwd  the window applied to those three derivative maps (the window
//               is symmetric, so it is its own adjoint) ->
//               dL/dx = (1 - lam) sign(x - y) / n - lam / n (G*A + 2 x G*B + y G*C).
#include "linprim_common.h"

namespace linprim {

constexpr int kSsimTile = 32;
constexpr int kSsimHalo = 5;
constexpr int kSsimIn = kSsimTile + 2 * kSsimHalo;   // 42
constexpr float kC1 = 0.0001f;                       // 0.01^2
constexpr float kC2 = 0.0009f;                       // 0.03^2

struct SsimWindow {
    float w[11];
};

// Loads 42 x 42 tiles of NT images (zero outside the image) into LDS.  All
// of a thread's global loads are issued before the first LDS store, so the
// block waits for memory once rather than once per element.
constexpr int kTileElems = kSsimIn * kSsimIn;             // 1764
constexpr int kLoadIters = (kTileElems + 255) / 256;      // 7 for 256 threads
template <int NT>
__device__ inline void load_tiles(const float* const (&src)[NT], int W, int H, int x0, int y0,
                                  float* const (&dst)[NT]) {
    float v[NT][kLoadIters];
#pragma unroll
    for (int it = 0; it < kLoadIters; ++it) {
        const int k = (int)threadIdx.x + it * 256;
        const int r = k / kSsimIn, c = k - r * kSsimIn;
        const int y = y0 - kSsimHalo + r, x = x0 - kSsimHalo + c;
        const bool in = k < kTileElems && x >= 0 && x < W && y >= 0 && y < H;
        const int64_t off = in ? (int64_t)y * W + x : 0;
#pragma unroll
        for (int m = 0; m < NT; ++m) v[m][it] = in ? src[m][off] : 0.0f;
    }
#pragma unroll
    for (int it = 0; it < kLoadIters; ++it) {
        const int k = (int)threadIdx.x + it * 256;
        if (k < kTileElems) {
#pragma unroll
            for (int m = 0; m < NT; ++m) dst[m][k] = v[m][it];
        }
    }
}

__global__ __launch_bounds__(256) void k_ssim_fwd(const float* __restrict__ rgb, const float* __restrict__ target,
                                                  int W, int H, SsimWindow win, float* __restrict__ dmaps,
                                                  float* __restrict__ partial, const uint32_t* __restrict__ skip) {
    if (skip && *skip) return;
    __shared__ float xs[kSsimIn * kSsimIn], ys[kSsimIn * kSsimIn];
    __shared__ float hs[5][kSsimIn * kSsimTile];
    __shared__ float red[2][256];
    const int ch = blockIdx.z;
    const int x0 = blockIdx.x * kSsimTile, y0 = blockIdx.y * kSsimTile;
    const int64_t hw = (int64_t)W * H;
    const float* X = rgb + ch * hw;
    const float* Y = target + ch * hw;
    {
        const float* const srcs[2] = {X, Y};
        float* const dsts[2] = {xs, ys};
        load_tiles<2>(srcs, W, H, x0, y0, dsts);
    }
    __syncthreads();
    // row pass: 42 rows x 32 output columns, five statistics; a thread
    // takes 4 neighbouring outputs of a row and slides over 14 inputs
    constexpr int RUN = 4, NRUN = kSsimTile / RUN;     // 8 runs per row
    for (int k = threadIdx.x; k < kSsimIn * NRUN; k += 256) {
        const int r = k / NRUN, c0 = (k % NRUN) * RUN;
        float acc[5][RUN];
#pragma unroll
        for (int q = 0; q < RUN; ++q)
#pragma unroll
            for (int m = 0; m < 5; ++m) acc[m][q] = 0.f;
#pragma unroll
        for (int i = 0; i < RUN + 10; ++i) {
            const float xv = xs[r * kSsimIn + c0 + i], yv = ys[r * kSsimIn + c0 + i];
            const float xx = xv * xv, yy = yv * yv, xy = xv * yv;
#pragma unroll
            for (int q = 0; q < RUN; ++q) {
                const int u = i - q;     // tap of output c0 + q
                if (u < 0 || u > 10) continue;
                const float wt = win.w[u];
                acc[0][q] += wt * xv;
                acc[1][q] += wt * yv;
                acc[2][q] += wt * xx;
                acc[3][q] += wt * yy;
                acc[4][q] += wt * xy;
            }
        }
#pragma unroll
        for (int q = 0; q < RUN; ++q)
#pragma unroll
            for (int m = 0; m < 5; ++m) hs[m][r * kSsimTile + c0 + q] = acc[m][q];
    }
    __syncthreads();
    // column pass: a thread takes 4 neighbouring rows of one column
    // (lanes run along a row, so the map stores are coalesced)
    float ssum = 0.f, l1 = 0.f;
    {
        const int c = threadIdx.x % kSsimTile, r0 = (threadIdx.x / kSsimTile) * RUN;   // 8 x 4 rows
        float acc[5][RUN];
#pragma unroll
        for (int q = 0; q < RUN; ++q)
#pragma unroll
            for (int m = 0; m < 5; ++m) acc[m][q] = 0.f;
#pragma unroll
        for (int i = 0; i < RUN + 10; ++i) {
            float v[5];
#pragma unroll
            for (int m = 0; m < 5; ++m) v[m] = hs[m][(r0 + i) * kSsimTile + c];
#pragma unroll
            for (int q = 0; q < RUN; ++q) {
                const int u = i - q;
                if (u < 0 || u > 10) continue;
                const float wt = win.w[u];
#pragma unroll
                for (int m = 0; m < 5; ++m) acc[m][q] += wt * v[m];
            }
        }
        float* dm = dmaps + (int64_t)ch * 3 * hw;
#pragma unroll
        for (int q = 0; q < RUN; ++q) {
            const int r = r0 + q;
            const int x = x0 + c, y = y0 + r;
            if (x >= W || y >= H) continue;
            const float mx = acc[0][q], my = acc[1][q], exx = acc[2][q], eyy = acc[3][q], exy = acc[4][q];
            const float A = 2.f * mx * my + kC1;
            const float B = 2.f * (exy - mx * my) + kC2;
            const float Cc = mx * mx + my * my + kC1;
            const float D = (exx - mx * mx) + (eyy - my * my) + kC2;
            const float icd = 1.0f / (Cc * D);
            const float sv = A * B * icd;
            const int64_t p = (int64_t)y * W + x;
            dm[p] = 2.f * my * (B - A) * icd - 2.f * mx * sv / Cc + 2.f * mx * sv / D;   // ds/dmx
            dm[hw + p] = -sv / D;                                                       // ds/dE[x^2]
            dm[2 * hw + p] = 2.f * A * icd;                                            // ds/dE[xy]
            ssum += sv;
            l1 += fabsf(xs[(r + kSsimHalo) * kSsimIn + c + kSsimHalo] - ys[(r + kSsimHalo) * kSsimIn + c + kSsimHalo]);
        }
    }
    // block sums, fixed order
    red[0][threadIdx.x] = ssum;
    red[1][threadIdx.x] = l1;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) {
            red[0][threadIdx.x] += red[0][threadIdx.x + off];
            red[1][threadIdx.x] += red[1][threadIdx.x + off];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const int64_t b = ((int64_t)ch * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
        partial[2 * b] = red[0][0];
        partial[2 * b + 1] = red[1][0];
    }
}

__global__ __launch_bounds__(256) void k_ssim_bwd(const float* __restrict__ rgb, const float* __restrict__ target,
                                                  int W, int H, SsimWindow win, const float* __restrict__ dmaps,
                                                  float l1_scale, float ssim_scale, float* __restrict__ grad,
                                                  const uint32_t* __restrict__ skip) {
    if (skip && *skip) return;
    __shared__ float ts[3][kSsimIn * kSsimIn];
    __shared__ float hs[3][kSsimIn * kSsimTile];
    const int ch = blockIdx.z;
    const int x0 = blockIdx.x * kSsimTile, y0 = blockIdx.y * kSsimTile;
    const int64_t hw = (int64_t)W * H;
    const float* dm = dmaps + (int64_t)ch * 3 * hw;
    {
        const float* const srcs[3] = {dm, dm + hw, dm + 2 * hw};
        float* const dsts[3] = {ts[0], ts[1], ts[2]};
        load_tiles<3>(srcs, W, H, x0, y0, dsts);
    }
    __syncthreads();
    // row pass over the three maps, 4 outputs per thread (sliding window)
    constexpr int RUN = 4, NRUN = kSsimTile / RUN;
    for (int k = threadIdx.x; k < kSsimIn * NRUN; k += 256) {
        const int r = k / NRUN, c0 = (k % NRUN) * RUN;
        float acc[3][RUN];
#pragma unroll
        for (int q = 0; q < RUN; ++q)
#pragma unroll
            for (int m = 0; m < 3; ++m) acc[m][q] = 0.f;
#pragma unroll
        for (int i = 0; i < RUN + 10; ++i) {
            float v[3];
#pragma unroll
            for (int m = 0; m < 3; ++m) v[m] = ts[m][r * kSsimIn + c0 + i];
#pragma unroll
            for (int q = 0; q < RUN; ++q) {
                const int u = i - q;
                if (u < 0 || u > 10) continue;
                const float wt = win.w[u];
#pragma unroll
                for (int m = 0; m < 3; ++m) acc[m][q] += wt * v[m];
            }
        }
#pragma unroll
        for (int q = 0; q < RUN; ++q)
#pragma unroll
            for (int m = 0; m < 3; ++m) hs[m][r * kSsimTile + c0 + q] = acc[m][q];
    }
    __syncthreads();
    const float* X = rgb + ch * hw;
    const float* Y = target + ch * hw;
    float* G = grad + ch * hw;
    // column pass: 4 neighbouring rows of one column per thread
    const int c = threadIdx.x % kSsimTile, r0 = (threadIdx.x / kSsimTile) * RUN;
    float acc[3][RUN];
#pragma unroll
    for (int q = 0; q < RUN; ++q)
#pragma unroll
        for (int m = 0; m < 3; ++m) acc[m][q] = 0.f;
#pragma unroll
    for (int i = 0; i < RUN + 10; ++i) {
        float v[3];
#pragma unroll
        for (int m = 0; m < 3; ++m) v[m] = hs[m][(r0 + i) * kSsimTile + c];
#pragma unroll
        for (int q = 0; q < RUN; ++q) {
            const int u = i - q;
            if (u < 0 || u > 10) continue;
            const float wt = win.w[u];
#pragma unroll
            for (int m = 0; m < 3; ++m) acc[m][q] += wt * v[m];
        }
    }
#pragma unroll
    for (int q = 0; q < RUN; ++q) {
        const int x = x0 + c, y = y0 + r0 + q;
        if (x >= W || y >= H) continue;
        const int64_t p = (int64_t)y * W + x;
        const float xv = X[p], yv = Y[p];
        const float d = xv - yv;
        const float sg = d > 0.f ? 1.f : (d < 0.f ? -1.f : 0.f);
        G[p] = l1_scale * sg - ssim_scale * (acc[0][q] + 2.f * xv * acc[1][q] + yv * acc[2][q]);
    }
}

SsimWindow ssim_window() {
    SsimWindow S;
    double g[11], tot = 0.0;
    for (int t = 0; t < 11; ++t) {
        const double r = t - 5;
        g[t] = exp(-(r * r) / (2.0 * 1.5 * 1.5));
        tot += g[t];
    }
    for (int t = 0; t < 11; ++t) S.w[t] = (float)(g[t] / tot);
    return S;
}

// One view [3, H, W]: dmaps [3][3][H][W] scratch, partial [2 * 3 * tiles].
hipError_t launch_ssim_l1(const float* rgb, const float* target, int W, int H, float lam, float* dmaps,
                          float* partial, float* grad, const uint32_t* skip, hipStream_t s) {
    const SsimWindow win = ssim_window();
    const dim3 grid((unsigned)((W + kSsimTile - 1) / kSsimTile), (unsigned)((H + kSsimTile - 1) / kSsimTile), 3);
    hipLaunchKernelGGL(k_ssim_fwd, grid, dim3(256), 0, s, rgb, target, W, H, win, dmaps, partial, skip);
    const float n = 3.0f * (float)W * (float)H;
    hipLaunchKernelGGL(k_ssim_bwd, grid, dim3(256), 0, s, rgb, target, W, H, win, dmaps, (1.0f - lam) / n, lam / n,
                       grad, skip);
    return hipGetLastError();
}

}  // namespace linprim
