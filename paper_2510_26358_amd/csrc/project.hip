// Projection of 3D Gaussians into every view of the batch (forward).
//
// One thread per Gaussian reads its parameters once (coalesced structure-of-arrays loads)
// and loops over the views whose Gaussian range contains it, so a rig of B cameras costs
// one parameter read instead of B.  Per view it computes (Sec. III-B):
//   x_c = R_b mu + t_b (in float64, rounded once); Sigma = R(q) diag(e^{2s}) R(q)^T;
//   Sigma' = J R_b Sigma R_b^T J^T + blur I; conic = Sigma'^{-1};
//   (u, v) = (fx x/z + cx, fy y/z + cy); o = sigmoid(omega);
//   colour = max(0, SH(d) . f + 0.5) with d the unit direction from the camera centre;
//   opacity-aware footprint half-extents ex = sqrt(2 ln(o / alpha_min) Sigma'_xx), ey likewise
//   (the box outside which alpha < alpha_min), the tile rectangle and its tile count; a kept pair's
//   row of the backward's 2D adjoint accumulator is zeroed.
// Culled pairs (z < z_near, det <= 0, o < alpha_min, empty rectangle) get count 0 and no
// record.
// The SH coefficients (48 of the 59 floats at degree 3) are read once per Gaussian that
// some view keeps: a first pass over the views writes the geometry part of each record, a
// second pass over the views that keep the Gaussian evaluates the colour.  (Reading them in
// the view loop fetched each cache line once per view.)
#include "common.h"

namespace ags {

template <int DEG>
__global__ __launch_bounds__(256) void project_fwd_kernel(ProjectArgs a) {
    constexpr int K = (DEG + 1) * (DEG + 1);
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.n) return;
    const int n = a.n;
    const ViewTable& vt = a.vt;

    const float mx = a.means[i], my = a.means[n + i], mz = a.means[2 * n + i];
    const float o = 1.f / (1.f + __expf(-a.logits[i]));
    const bool o_ok = o >= a.st.alpha_min;

    float s0 = __expf(a.log_scales[i]), s1 = __expf(a.log_scales[n + i]), s2 = __expf(a.log_scales[2 * n + i]);
    float qw = a.quats[i], qx = a.quats[n + i], qy = a.quats[2 * n + i], qz = a.quats[3 * n + i];
    float qinv = rsqrtf(qw * qw + qx * qx + qy * qy + qz * qz);
    qw *= qinv; qx *= qinv; qy *= qinv; qz *= qinv;
    float Rq[9];
    quat_to_rot(qw, qx, qy, qz, Rq);
    // M = Rq diag(s); Sigma = M M^T (symmetric: 6 entries)
    float M[9] = {Rq[0] * s0, Rq[1] * s1, Rq[2] * s2, Rq[3] * s0, Rq[4] * s1, Rq[5] * s2,
                  Rq[6] * s0, Rq[7] * s1, Rq[8] * s2};
    const float S00 = M[0] * M[0] + M[1] * M[1] + M[2] * M[2];
    const float S01 = M[0] * M[3] + M[1] * M[4] + M[2] * M[5];
    const float S02 = M[0] * M[6] + M[1] * M[7] + M[2] * M[8];
    const float S11 = M[3] * M[3] + M[4] * M[4] + M[5] * M[5];
    const float S12 = M[3] * M[6] + M[4] * M[7] + M[5] * M[8];
    const float S22 = M[6] * M[6] + M[7] * M[7] + M[8] * M[8];
    const float lnterm = 2.f * __logf(o / a.st.alpha_min);

    uint32_t vis = 0;  // views that keep this Gaussian (at most 32)
    for (int b = 0; b < vt.n_views; ++b) {
        if (i < vt.g_begin[b] || i >= vt.g_end[b]) continue;
        const long long q = vt.pair_base[b] + (i - vt.g_begin[b]);
        const ags_camera cam = a.cams[b];
        const float* R = cam.R;
        float x, y, z;
        world_to_cam(cam, mx, my, mz, x, y, z);
        uint32_t cnt = 0;
        if (o_ok && z >= a.st.z_near) {
            const int W = vt.width[b], H = vt.height[b];
            const float rz = 1.f / z;
            const float limx = a.st.fov_clamp * (float)W / (2.f * cam.fx);
            const float limy = a.st.fov_clamp * (float)H / (2.f * cam.fy);
            const float txz = fminf(fmaxf(x * rz, -limx), limx);
            const float tyz = fminf(fmaxf(y * rz, -limy), limy);
            // J = [[fx/z, 0, -fx tx/z^2], [0, fy/z, -fy ty/z^2]] with tx = txz z
            const float j00 = cam.fx * rz, j02 = -cam.fx * txz * rz;
            const float j11 = cam.fy * rz, j12 = -cam.fy * tyz * rz;
            // T = J R (2x3)
            const float T0[3] = {j00 * R[0] + j02 * R[6], j00 * R[1] + j02 * R[7], j00 * R[2] + j02 * R[8]};
            const float T1[3] = {j11 * R[3] + j12 * R[6], j11 * R[4] + j12 * R[7], j11 * R[5] + j12 * R[8]};
            // Sigma' = T Sigma T^T
            const float u0 = S00 * T0[0] + S01 * T0[1] + S02 * T0[2];
            const float u1 = S01 * T0[0] + S11 * T0[1] + S12 * T0[2];
            const float u2 = S02 * T0[0] + S12 * T0[1] + S22 * T0[2];
            const float w0 = S00 * T1[0] + S01 * T1[1] + S02 * T1[2];
            const float w1 = S01 * T1[0] + S11 * T1[1] + S12 * T1[2];
            const float w2 = S02 * T1[0] + S12 * T1[1] + S22 * T1[2];
            const float ca = T0[0] * u0 + T0[1] * u1 + T0[2] * u2 + a.st.blur;
            const float cb = T1[0] * u0 + T1[1] * u1 + T1[2] * u2;
            const float cc = T1[0] * w0 + T1[1] * w1 + T1[2] * w2 + a.st.blur;
            const float det = ca * cc - cb * cb;
            if (det > 0.f) {
                const float idet = 1.f / det;
                const float u = cam.fx * x * rz + cam.cx;
                const float v = cam.fy * y * rz + cam.cy;
                const float ex = sqrtf(lnterm * ca);
                const float ey = sqrtf(lnterm * cc);
                int tx0, ty0, tx1, ty1;
                if (tile_rect(u, v, ex, ey, W, H, vt.tile, tx0, ty0, tx1, ty1)) {
                    cnt = (uint32_t)((tx1 - tx0 + 1) * (ty1 - ty0 + 1));
                    float4* rec = reinterpret_cast<float4*>(a.records + q * kRecFloats);
                    rec[0] = make_float4(u, v, cc * idet, -cb * idet);
                    rec[1] = make_float4(ca * idet, o, z, ex);
                    a.records[q * kRecFloats + 8] = ey;
                    a.pair_z[q] = __float_as_uint(z);
                    // the pair's 2D adjoint row starts the backward at zero
                    float4* row = reinterpret_cast<float4*>(a.grad2d + q * kGrad2dStride);
#pragma unroll
                    for (int c = 0; c < kGrad2dStride / 4; ++c) row[c] = make_float4(0.f, 0.f, 0.f, 0.f);
                    vis |= 1u << b;
                }
            }
        }
        a.pair_count[q] = cnt;
        if (!cnt) a.pair_z[q] = kNoDepth;  // dropped by the depth sort's first pass
    }
    if (vis == 0u) return;

    // colour: the coefficients once (the lanes of the wave that need them load together),
    // then each view that keeps the Gaussian
    float f[K][3];
#pragma unroll
    for (int k = 0; k < K; ++k)
#pragma unroll
        for (int c = 0; c < 3; ++c) f[k][c] = sh_row(a.sh, n, k * 3 + c)[(uint32_t)i];
    while (vis) {
        const int b = __builtin_ctz(vis);
        vis &= vis - 1u;
        const long long q = vt.pair_base[b] + (i - vt.g_begin[b]);
        const ags_camera cam = a.cams[b];
        // camera centre C = -R^T t; direction d = (mu - C) / |mu - C|
        float dx, dy, dz;
        centre_to_mean(cam, mx, my, mz, dx, dy, dz);
        const float il = rsqrtf(dx * dx + dy * dy + dz * dz);
        dx *= il; dy *= il; dz *= il;
        float Y[16];
        sh_basis(DEG, dx, dy, dz, Y);
        float col[3] = {0.f, 0.f, 0.f};
#pragma unroll
        for (int k = 0; k < K; ++k)
#pragma unroll
            for (int c = 0; c < 3; ++c) col[c] += Y[k] * f[k][c];
        float* rc = a.records + q * kRecFloats + 9;
        rc[0] = fmaxf(col[0] + 0.5f, 0.f);
        rc[1] = fmaxf(col[1] + 0.5f, 0.f);
        rc[2] = fmaxf(col[2] + 0.5f, 0.f);
    }
}

void launch_project_fwd(const ProjectArgs& a, hipStream_t s) {
    if (a.n <= 0) return;
    dim3 grid((a.n + 255) / 256), block(256);
    switch (a.sh_degree) {
        case 0: hipLaunchKernelGGL(project_fwd_kernel<0>, grid, block, 0, s, a); break;
        case 1: hipLaunchKernelGGL(project_fwd_kernel<1>, grid, block, 0, s, a); break;
        case 2: hipLaunchKernelGGL(project_fwd_kernel<2>, grid, block, 0, s, a); break;
        default: hipLaunchKernelGGL(project_fwd_kernel<3>, grid, block, 0, s, a); break;
    }
}

}  // namespace ags
