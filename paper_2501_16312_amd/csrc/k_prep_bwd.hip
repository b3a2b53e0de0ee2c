// k_prep_bwd.hip -- preprocessing backward pass (Sec. 3.4 "Preprocessing
// Backpropagation"): per primitive, sum its per-tile gradient records, then
// undo the plane construction, the ray-space projection and the view
// transform, and split the corner gradients onto rotation and distances.
// One thread per primitive loops over the views, so gradients summed over
// views are deterministic.  Double precision throughout (memory-bound).
#include "linprim_common.h"

namespace linprim {

struct V3 {
    double x, y, z;
};

__device__ inline void cross3(const double a[3], const double b[3], double o[3]) {
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
}

template <int KIND>
__global__ __launch_bounds__(128) void k_prep_bwd(const float* __restrict__ means, const float* __restrict__ quats,
                                                  const float* __restrict__ dists, const float* __restrict__ opacity,
                                                  const float* __restrict__ sh, int sh_degree, int64_t n, int n_views,
                                                  const ViewInfo* __restrict__ views, const float* __restrict__ payload,
                                                  const uint32_t* __restrict__ tiles,
                                                  const uint32_t* __restrict__ offsets,
                                                  const float* __restrict__ grads, const Status* __restrict__ status,
                                                  uint64_t capacity, float* __restrict__ g_means,
                                                  float* __restrict__ g_quats, float* __restrict__ g_dists,
                                                  float* __restrict__ g_opacity, float* __restrict__ g_sh) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    constexpr int ND = (KIND == LINPRIM_OCTAHEDRON) ? 3 : 4;
    const int K = (sh_degree + 1) * (sh_degree + 1);
    const bool ok = status->n_pairs <= capacity;
    double gm[3] = {0, 0, 0}, gq[4] = {0, 0, 0, 0}, gd[4] = {0, 0, 0, 0}, ga_total = 0.0;
    float* gsh = g_sh + i * (int64_t)K * 3;
    for (int k = 0; k < 3 * K; ++k) gsh[k] = 0.0f;
    for (int v = 0; ok && v < n_views; ++v) {
        const int64_t slot = (int64_t)v * n + i;
        const uint32_t cnt = tiles[slot];
        if (cnt == 0) continue;
        // sum of the per-tile records, in tile order
        double r[kGradWords];
        for (int k = 0; k < kGradWords; ++k) r[k] = 0.0;
        const float4* gp = reinterpret_cast<const float4*>(grads + (int64_t)offsets[slot] * kGradWords);
        for (uint32_t t = 0; t < cnt; ++t) {
#pragma unroll
            for (int k = 0; k < kGradWords / 4; ++k) {
                const float4 x = gp[(int64_t)t * (kGradWords / 4) + k];
                r[4 * k + 0] += x.x;
                r[4 * k + 1] += x.y;
                r[4 * k + 2] += x.z;
                r[4 * k + 3] += x.w;
            }
        }
        const ViewInfo& V = views[v];
        Geom G;
        if (!build_geometry(KIND, means + 3 * i, quats + 4 * i, dists + ND * i, opacity[i], V, G)) continue;
        const float* rec = payload + slot * kRecordWords;
        const int i0 = __float_as_int(rec[R_I0]), j0 = __float_as_int(rec[R_J0]);
        const double ox = (double)i0 + 0.5 - G.c[0];
        const double oy = (double)j0 + 0.5 - G.c[1];

        // ---- planes -> ray-space centre (xy) and offsets a_k
        double gox = 0.0, goy = 0.0;
        double ga[4][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
        if (KIND == LINPRIM_OCTAHEDRON) {
            double M[9], N[9], gN[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
            for (int rr = 0; rr < 3; ++rr)
                for (int k = 0; k < 3; ++k) M[3 * rr + k] = G.a[k][rr];
            inverse3(M, N);
            for (int s = 0; s < 4; ++s) {
                double nu[3];
                for (int c = 0; c < 3; ++c)
                    nu[c] = kSlab[s][0] * N[c] + kSlab[s][1] * N[3 + c] + kSlab[s][2] * N[6 + c];
                const double nl = sqrt(nu[0] * nu[0] + nu[1] * nu[1] + nu[2] * nu[2]);
                const double nz = clamp_nz(nu[2], nl);
                const double A = -nu[0] / nz, B = -nu[1] / nz, Wd = 1.0 / fabs(nz);
                const double gA = r[4 * s], gB = r[4 * s + 1], gUp = r[4 * s + 2], gLo = r[4 * s + 3];
                const double gsum = gUp + gLo;         // both offsets carry A ox + B oy
                const double gW = gUp - gLo;
                const double gAt = gA + gsum * ox, gBt = gB + gsum * oy;
                gox += gsum * A;
                goy += gsum * B;
                const double gnu0 = -gAt / nz, gnu1 = -gBt / nz;
                const double gnu2 = -(gAt * A + gBt * B + gW * Wd) / nz;
                for (int c = 0; c < 3; ++c) {
                    const double gn = (c == 0) ? gnu0 : (c == 1) ? gnu1 : gnu2;
                    gN[0 + c] += kSlab[s][0] * gn;
                    gN[3 + c] += kSlab[s][1] * gn;
                    gN[6 + c] += kSlab[s][2] * gn;
                }
            }
            // N = M^-1:  dL/dM = -N^T dL/dN N^T
            double T1[9];
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) {
                    double s = 0.0;
                    for (int c = 0; c < 3; ++c) s += N[3 * c + a] * gN[3 * c + b];
                    T1[3 * a + b] = s;     // N^T gN
                }
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) {
                    double s = 0.0;
                    for (int c = 0; c < 3; ++c) s += T1[3 * a + c] * N[3 * b + c];
                    // column b of M is a_b: gM[a][b] = dL/d a_b[a]
                    ga[b][a] = -s;
                }
        } else {
            for (int f = 0; f < 4; ++f) {
                const double gA = r[3 * f], gB = r[3 * f + 1], gDp = r[3 * f + 2];
                int m[3], q = 0;
                for (int k = 0; k < 4; ++k)
                    if (k != f) m[q++] = k;
                const double* P0 = G.a[m[0]];
                const double e1[3] = {G.a[m[1]][0] - P0[0], G.a[m[1]][1] - P0[1], G.a[m[1]][2] - P0[2]};
                const double e2[3] = {G.a[m[2]][0] - P0[0], G.a[m[2]][1] - P0[1], G.a[m[2]][2] - P0[2]};
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
                double gP0[3] = {-gDp * A, -gDp * B, gDp};
                gox += gDp * A;
                goy += gDp * B;
                double gn[3] = {-gAt / nz, -gBt / nz, -(gAt * A + gBt * B) / nz};
                for (int c = 0; c < 3; ++c) gn[c] *= sgn;     // gradient of e1 x e2
                double ge1[3], ge2[3];
                cross3(e2, gn, ge1);
                cross3(gn, e1, ge2);
                for (int c = 0; c < 3; ++c) {
                    ga[m[0]][c] += gP0[c] - ge1[c] - ge2[c];
                    ga[m[1]][c] += ge1[c];
                    ga[m[2]][c] += ge2[c];
                }
            }
        }
        // ox = i0 + 1/2 - c_x, oy = j0 + 1/2 - c_y
        const double gc[3] = {-gox, -goy, 0.0};

        // ---- ray space -> camera: c = phi(t) with d phi/dt = J; a_k = J(t) oc_k
        const double* J = G.J;
        const double x = G.tc[0], y = G.tc[1], z = G.tc[2];
        const double l = G.c[2];
        double gt[3];
        for (int c = 0; c < 3; ++c) gt[c] = J[c] * gc[0] + J[3 + c] * gc[1] + J[6 + c] * gc[2];
        double goc[4][3];
        for (int k = 0; k < ND; ++k) {
            for (int c = 0; c < 3; ++c) goc[k][c] = J[c] * ga[k][0] + J[3 + c] * ga[k][1] + J[6 + c] * ga[k][2];
            const double* w = G.oc[k];
            const double tw = x * w[0] + y * w[1] + z * w[2];
            const double l3 = l * l * l, z2 = z * z, z3 = z2 * z;
            // derivatives of J w with respect to t (rows: output, cols: t)
            const double d00 = -V.fx * w[2] / z2, d02 = -V.fx * w[0] / z2 + 2.0 * V.fx * x * w[2] / z3;
            const double d11 = -V.fy * w[2] / z2, d12 = -V.fy * w[1] / z2 + 2.0 * V.fy * y * w[2] / z3;
            const double d20 = w[0] / l - tw * x / l3, d21 = w[1] / l - tw * y / l3, d22 = w[2] / l - tw * z / l3;
            gt[0] += d00 * ga[k][0] + d20 * ga[k][2];
            gt[1] += d11 * ga[k][1] + d21 * ga[k][2];
            gt[2] += d02 * ga[k][0] + d12 * ga[k][1] + d22 * ga[k][2];
        }
        // ---- camera -> world
        for (int c = 0; c < 3; ++c) gm[c] += V.Rw[c] * gt[0] + V.Rw[3 + c] * gt[1] + V.Rw[6 + c] * gt[2];
        double gR[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
        for (int k = 0; k < ND; ++k) {
            double go[3];
            for (int c = 0; c < 3; ++c) go[c] = V.Rw[c] * goc[k][0] + V.Rw[3 + c] * goc[k][1] + V.Rw[6 + c] * goc[k][2];
            if (KIND == LINPRIM_OCTAHEDRON) {
                const double dk = (double)dists[ND * i + k];
                double dd = 0.0;
                for (int rr = 0; rr < 3; ++rr) {
                    gR[3 * rr + k] += go[rr] * dk;
                    dd += go[rr] * G.R[3 * rr + k];
                }
                gd[k] += dd;
            } else {
                const double gk = (double)dists[ND * i + k] * kInvSqrt3;
                double dd = 0.0;
                for (int rr = 0; rr < 3; ++rr) {
                    const double rb = kTetDir[k][0] * G.R[3 * rr] + kTetDir[k][1] * G.R[3 * rr + 1] +
                                      kTetDir[k][2] * G.R[3 * rr + 2];
                    for (int c = 0; c < 3; ++c) gR[3 * rr + c] += go[rr] * kTetDir[k][c] * gk;
                    dd += go[rr] * rb * kInvSqrt3;
                }
                gd[k] += dd;
            }
        }
        // ---- rotation -> quaternion through R = I + s K(q), s = 2/|q|^2
        {
            const double w = quats[4 * i], qx = quats[4 * i + 1], qy = quats[4 * i + 2], qz = quats[4 * i + 3];
            const double n2 = w * w + qx * qx + qy * qy + qz * qz;
            const double s = 2.0 / n2;
            const double Km[9] = {-(qy * qy + qz * qz), qx * qy - w * qz, qx * qz + w * qy,
                                  qx * qy + w * qz, -(qx * qx + qz * qz), qy * qz - w * qx,
                                  qx * qz - w * qy, qy * qz + w * qx, -(qx * qx + qy * qy)};
            double gK = 0.0;
            for (int k = 0; k < 9; ++k) gK += gR[k] * Km[k];
            const double qv[4] = {w, qx, qy, qz};
            // dK/dw, dK/dx, dK/dy, dK/dz
            const double dK[4][9] = {{0, -qz, qy, qz, 0, -qx, -qy, qx, 0},
                                     {0, qy, qz, qy, -2 * qx, -w, qz, w, -2 * qx},
                                     {-2 * qy, qx, w, qx, 0, qz, -w, qz, -2 * qy},
                                     {-2 * qz, -w, qx, w, -2 * qz, qy, qx, qy, 0}};
            for (int mm = 0; mm < 4; ++mm) {
                double acc = -s * s * qv[mm] * gK;
                for (int k = 0; k < 9; ++k) acc += s * gR[k] * dK[mm][k];
                gq[mm] += acc;
            }
        }
        // ---- Eq. 1 with min(d) held constant
        {
            double dmin = (double)dists[ND * i];
            for (int k = 1; k < ND; ++k) dmin = fmin(dmin, (double)dists[ND * i + k]);
            const double al = (double)opacity[i];
            ga_total += r[19] * kAlphaScaleD / ((1.0 - kAlphaScaleD * al) * 2.0 * dmin);
        }
        // ---- colour -> SH coefficients and viewing direction
        {
            double dir[3] = {(double)means[3 * i] - V.cam_pos[0], (double)means[3 * i + 1] - V.cam_pos[1],
                             (double)means[3 * i + 2] - V.cam_pos[2]};
            const double dn = sqrt(dir[0] * dir[0] + dir[1] * dir[1] + dir[2] * dir[2]);
            for (int c = 0; c < 3; ++c) dir[c] /= dn;
            double Y[16], GY[16][3];
            sh_eval(sh_degree, dir[0], dir[1], dir[2], Y);
            sh_eval_grad(sh_degree, dir[0], dir[1], dir[2], GY);
            const float* shp = sh + i * (int64_t)K * 3;
            double gdir[3] = {0, 0, 0};
            for (int ch = 0; ch < 3; ++ch) {
                double raw = 0.5;
                for (int k = 0; k < K; ++k) raw += (double)shp[3 * k + ch] * Y[k];
                if (!(raw > 0.0)) continue;
                const double gr = r[16 + ch];
                for (int k = 0; k < K; ++k) {
                    gsh[3 * k + ch] += (float)(gr * Y[k]);
                    for (int c = 0; c < 3; ++c) gdir[c] += gr * (double)shp[3 * k + ch] * GY[k][c];
                }
            }
            const double dot = gdir[0] * dir[0] + gdir[1] * dir[1] + gdir[2] * dir[2];
            for (int c = 0; c < 3; ++c) gm[c] += (gdir[c] - dot * dir[c]) / dn;
        }
    }
    for (int c = 0; c < 3; ++c) g_means[3 * i + c] = (float)gm[c];
    for (int c = 0; c < 4; ++c) g_quats[4 * i + c] = (float)gq[c];
    for (int c = 0; c < ND; ++c) g_dists[ND * i + c] = (float)gd[c];
    g_opacity[i] = (float)ga_total;
}

hipError_t launch_preprocess_bwd(const linprim_prims& p, int32_t n_views, int tile, const ViewLayout& L,
                                 const char* vws, const PairLayout& P, const char* pws, float* g_means,
                                 float* g_quats, float* g_dists, float* g_opacity, float* g_sh, hipStream_t stream) {
    (void)tile;
    if (p.n == 0) return hipSuccess;
    const ViewInfo* views = reinterpret_cast<const ViewInfo*>(vws + L.views);
    const float* payload = reinterpret_cast<const float*>(vws + L.payload);
    const uint32_t* tiles = reinterpret_cast<const uint32_t*>(vws + L.tiles);
    const uint32_t* offsets = reinterpret_cast<const uint32_t*>(vws + L.offsets);
    const Status* st = reinterpret_cast<const Status*>(vws + L.status);
    const float* grads = reinterpret_cast<const float*>(pws + P.grads);
    dim3 grid((unsigned)((p.n + 127) / 128));
    if (p.type == LINPRIM_OCTAHEDRON)
        hipLaunchKernelGGL(k_prep_bwd<LINPRIM_OCTAHEDRON>, grid, dim3(128), 0, stream, p.means, p.quats, p.dists, p.opacity,
                           p.sh, p.sh_degree, p.n, n_views, views, payload, tiles, offsets, grads, st,
                           (uint64_t)P.capacity, g_means, g_quats, g_dists, g_opacity, g_sh);
    else
        hipLaunchKernelGGL(k_prep_bwd<LINPRIM_TETRAHEDRON>, grid, dim3(128), 0, stream, p.means, p.quats, p.dists,
                           p.opacity, p.sh, p.sh_degree, p.n, n_views, views, payload, tiles, offsets, grads, st,
                           (uint64_t)P.capacity, g_means, g_quats, g_dists, g_opacity, g_sh);
    return hipGetLastError();
}

}  // namespace linprim
