// k_optim.hip -- the optimisation step around the rasterizer (Sec. 3.4
// "Optimization"): the L1 photometric loss gradient and a fused Adam update
// of every primitive feature in one launch.
#include "linprim_common.h"

namespace linprim {

// dL/dC = sign(C - target) * scale, with L = scale * sum |C - target|;
// per-block partial sums of |C - target| go to partial[blockIdx.x].
__global__ __launch_bounds__(256) void k_l1_grad(const float* __restrict__ rgb, const float* __restrict__ target,
                                                 int64_t count, float scale, float* __restrict__ grad,
                                                 float* __restrict__ partial) {
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

// One thread per 4 consecutive elements of the concatenated groups.
__global__ __launch_bounds__(256) void k_adam(AdamGroups G, float beta1, float beta2, float eps, float bc1_arg,
                                              float bc2_arg, const float* __restrict__ bias_corr) {
    const float bc1 = bias_corr ? bias_corr[0] : bc1_arg;
    const float bc2 = bias_corr ? bias_corr[1] : bc2_arg;
    const int64_t e0 = ((int64_t)blockIdx.x * 256 + threadIdx.x) * 4;
    if (e0 >= G.start[G.count]) return;
    int gi = 0;
    while (gi + 1 < G.count && G.start[gi + 1] <= e0) ++gi;
    for (int k = 0; k < 4; ++k) {
        const int64_t e = e0 + k;
        while (gi + 1 < G.count && G.start[gi + 1] <= e) ++gi;
        if (e >= G.start[G.count]) break;
        const int64_t i = e - G.start[gi];
        const float g = G.grad[gi][i];
        const float m = beta1 * G.m[gi][i] + (1.0f - beta1) * g;
        const float v = beta2 * G.v[gi][i] + (1.0f - beta2) * g * g;
        G.m[gi][i] = m;
        G.v[gi][i] = v;
        const float mh = m / bc1, vh = v / bc2;
        float p = G.param[gi][i] - G.lr[gi] * mh / (sqrtf(vh) + eps);
        p = fminf(fmaxf(p, G.lo[gi]), G.hi[gi]);
        G.param[gi][i] = p;
    }
}

hipError_t launch_l1_grad(const float* rgb, const float* target, int64_t count, float scale, float* grad,
                          float* partial, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    const int64_t blocks = (count + 1023) / 1024;
    hipLaunchKernelGGL(k_l1_grad, dim3((unsigned)blocks), dim3(256), 0, s, rgb, target, count, scale, grad, partial);
    return hipGetLastError();
}

hipError_t launch_adam(const AdamGroups& G, float beta1, float beta2, float eps, float bc1, float bc2,
                       const float* bias_corr, hipStream_t s) {
    const int64_t total = G.start[G.count];
    if (total <= 0) return hipSuccess;
    const int64_t blocks = (total + 1023) / 1024;
    hipLaunchKernelGGL(k_adam, dim3((unsigned)blocks), dim3(256), 0, s, G, beta1, beta2, eps, bc1, bc2, bias_corr);
    return hipGetLastError();
}

}  // namespace linprim
