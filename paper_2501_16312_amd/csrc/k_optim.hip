// k_optim.hip -- the optimisation step around the rasterizer (Sec. 3.4
// "Optimization"): the L1 photometric loss gradient and a fused Adam update
// of every primitive feature in one launch.
#include "linprim_common.h"

namespace linprim {

// dL/dC = sign(C - target) * scale, with L = scale * sum |C - target|;
// per-block partial sums of |C - target| go to partial[blockIdx.x].
__global__ __launch_bounds__(256) void k_l1_grad(const float* __restrict__ rgb, const float* __restrict__ target,
                                                 int64_t count, float scale, float* __restrict__ grad,
                                                 float* __restrict__ partial, const uint32_t* __restrict__ skip) {
    if (skip && *skip) return;
    __shared__ float red[4];
    const int64_t i0 = ((int64_t)blockIdx.x * 256 + threadIdx.x) * 4;
    float s = 0.0f;
    if (i0 + 3 < count) {
        const float4 c = *reinterpret_cast<const float4*>(rgb + i0);
        const float4 t = *reinterpret_cast<const float4*>(target + i0);
        const float d0 = c.x - t.x, d1 = c.y - t.y, d2 = c.z - t.z, d3 = c.w - t.w;
        auto sg = [](float d) { return d > 0.0f ? 1.0f : (d < 0.0f ? -1.0f : 0.0f); };
        *reinterpret_cast<float4*>(grad + i0) =
            make_float4(sg(d0) * scale, sg(d1) * scale, sg(d2) * scale, sg(d3) * scale);
        s = fabsf(d0) + fabsf(d1) + fabsf(d2) + fabsf(d3);
    } else {
        for (int64_t i = i0; i < count; ++i) {
            const float d = rgb[i] - target[i];
            grad[i] = (d > 0.0f ? 1.0f : (d < 0.0f ? -1.0f : 0.0f)) * scale;
            s += fabsf(d);
        }
    }
    for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) partial[blockIdx.x] = (red[0] + red[1] + red[2] + red[3]) * scale;
}

constexpr int kAdamBlock = 256;
constexpr int kAdamPerThread = 4;

__device__ inline void adam_one(float& p, float& m, float& v, float g, float lr, float beta1, float beta2, float eps,
                                float bc1, float bc2, float lo, float hi) {
    m = beta1 * m + (1.0f - beta1) * g;
    v = beta2 * v + (1.0f - beta2) * g * g;
    const float mh = m / bc1, vh = v / bc2;
    p = fminf(fmaxf(p - lr * mh / (sqrtf(vh) + eps), lo), hi);
}

// Each group owns a contiguous range of blocks; a thread updates 4
// consecutive elements of its group (one 16-byte access per array when the
// group's arrays are aligned).
__global__ __launch_bounds__(kAdamBlock) void k_adam(AdamGroups G, float beta1, float beta2, float eps, float bc1_arg,
                                                     float bc2_arg, const float* __restrict__ bias_corr,
                                                     const uint32_t* __restrict__ skip) {
    if (skip && *skip) return;
    const float bc1 = bias_corr ? bias_corr[0] : bc1_arg;
    const float bc2 = bias_corr ? bias_corr[1] : bc2_arg;
    int gi = 0;
    while (gi + 1 < G.count && G.block0[gi + 1] <= (int64_t)blockIdx.x) ++gi;
    const int64_t n = G.numel[gi];
    const int64_t e0 = (((int64_t)blockIdx.x - G.block0[gi]) * kAdamBlock + threadIdx.x) * kAdamPerThread;
    if (e0 >= n) return;
    float* __restrict__ P = G.param[gi];
    const float* __restrict__ Gr = G.grad[gi];
    float* __restrict__ M = G.m[gi];
    float* __restrict__ V = G.v[gi];
    const float lo = G.lo[gi], hi = G.hi[gi];
    const int period = G.period[gi], head = G.head[gi];
    float lr[kAdamPerThread];
#pragma unroll
    for (int k = 0; k < kAdamPerThread; ++k)
        lr[k] = (period > 0 && (int)((e0 + k) % period) >= head) ? G.lr_tail[gi] : G.lr[gi];
    if (G.vec[gi] && e0 + kAdamPerThread <= n) {
        float4 p = *reinterpret_cast<const float4*>(P + e0);
        const float4 g = *reinterpret_cast<const float4*>(Gr + e0);
        float4 m = *reinterpret_cast<const float4*>(M + e0);
        float4 v = *reinterpret_cast<const float4*>(V + e0);
        adam_one(p.x, m.x, v.x, g.x, lr[0], beta1, beta2, eps, bc1, bc2, lo, hi);
        adam_one(p.y, m.y, v.y, g.y, lr[1], beta1, beta2, eps, bc1, bc2, lo, hi);
        adam_one(p.z, m.z, v.z, g.z, lr[2], beta1, beta2, eps, bc1, bc2, lo, hi);
        adam_one(p.w, m.w, v.w, g.w, lr[3], beta1, beta2, eps, bc1, bc2, lo, hi);
        *reinterpret_cast<float4*>(P + e0) = p;
        *reinterpret_cast<float4*>(M + e0) = m;
        *reinterpret_cast<float4*>(V + e0) = v;
    } else {
        for (int k = 0; k < kAdamPerThread && e0 + k < n; ++k) {
            float p = P[e0 + k], m = M[e0 + k], v = V[e0 + k];
            adam_one(p, m, v, Gr[e0 + k], lr[k], beta1, beta2, eps, bc1, bc2, lo, hi);
            P[e0 + k] = p;
            M[e0 + k] = m;
            V[e0 + k] = v;
        }
    }
}

hipError_t launch_l1_grad(const float* rgb, const float* target, int64_t count, float scale, float* grad,
                          float* partial, const uint32_t* skip, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    const int64_t blocks = (count + 1023) / 1024;
    hipLaunchKernelGGL(k_l1_grad, dim3((unsigned)blocks), dim3(256), 0, s, rgb, target, count, scale, grad, partial,
                       skip);
    return hipGetLastError();
}

hipError_t launch_adam(const AdamGroups& G, float beta1, float beta2, float eps, float bc1, float bc2,
                       const float* bias_corr, const uint32_t* skip, hipStream_t s) {
    const int64_t blocks = G.block0[G.count];
    if (blocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_adam, dim3((unsigned)blocks), dim3(kAdamBlock), 0, s, G, beta1, beta2, eps, bc1, bc2,
                       bias_corr, skip);
    return hipGetLastError();
}

// Step guard of a captured training step: guard[0] = this step's
// pair-overflow flag, guard[1] |= it (cleared only by the caller).
__global__ void k_step_guard(const Status* __restrict__ status, uint32_t* __restrict__ guard) {
    if (threadIdx.x == 0) {
        const uint32_t ov = status->overflow ? 1u : 0u;
        guard[0] = ov;
        guard[1] |= ov;
    }
}

hipError_t launch_step_guard(const void* view_ws, const ViewLayout& L, uint32_t* guard, hipStream_t s) {
    const Status* st = reinterpret_cast<const Status*>((const char*)view_ws + L.status);
    hipLaunchKernelGGL(k_step_guard, dim3(1), dim3(64), 0, s, st, guard);
    return hipGetLastError();
}

}  // namespace linprim
