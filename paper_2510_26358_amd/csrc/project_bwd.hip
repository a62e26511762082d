// Adjoint of the projection (Sec. III-B) for every view, summed over views per Gaussian,
// plus each view's SE(3) pose adjoint (poses refined through the projection, Sec. III-C).
//
// One thread per Gaussian loops over the views that see it (the same splat set is shared
// by all cameras, so its gradient is the sum over views), reads the pair's ten 2D adjoints
// (u, v, conic a b c, opacity, depth), recomputes the forward quantities and chains:
//   conic -> Sigma':     G' = -K G_K K, G_K = [[ga, gb/2], [gb/2, gc]]
//   Sigma' = T Sigma T^T with T = J R_b:  G_Sigma += T^T G' T,  G_T = 2 G' T Sigma
//   T -> J -> x_c (x/z, y/z clamp: zero through the clamped coordinate), (u, v) -> x_c,
//   depth z -> x_c;  mu <- R_b^T g_xc.
// Pose, left perturbation W_b <- Exp(delta) W_b with delta = (rho, phi):
//   g_rho += g_xc,  g_phi += x_c x g_xc + (N_12 - N_21, N_20 - N_02, N_01 - N_10),
//   N = R_b G_T^T J.
// The colour part follows in the same kernel (a second phase of the thread, so the pair's
// 2D adjoint and the Gaussian's mean are still cached) and reads the SH coefficients once per
// Gaussian: the clamp-masked colour adjoint (the mask is the forward's stored colour > 0),
// Y(d) for the coefficients, and grad Y projected on the sphere for the direction
// d = (mu - C_b) / |mu - C_b|, which adds to mu and, through the camera centre moving by
// -R_b^T rho, g_rho += R_b g_dir.
// The per-view pose sums are reduced over the wave, then over the workgroup in LDS, into
// one partial per workgroup and view (one per phase); a second kernel adds the partials in a
// fixed order (deterministic, and no contention on the 6 B floats).  Shared-Gaussian terms
// (Sigma -> scale, rotation; opacity -> logit) are chained once after the view loop.
#include "common.h"

namespace ags {

void launch_project_bwd_main(const ProjectBwdArgs& a, hipStream_t s);

template <int DEG>
__device__ __forceinline__ void geometry_bwd(const ProjectBwdArgs& a) {
    constexpr int K = (DEG + 1) * (DEG + 1);
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const bool active = i < a.n;
    const int n = a.n;
    const int lane = __lane_id();
    const int wave = threadIdx.x >> 6;
    const ViewTable& vt = a.vt;
    __shared__ float spose[kMaxViews][6][4];
    for (int t = threadIdx.x; t < kMaxViews * 6 * 4; t += 256) (&spose[0][0][0])[t] = 0.f;
    __syncthreads();

    float mx = 0.f, my = 0.f, mz = 0.f, ls0 = 0.f, ls1 = 0.f, ls2 = 0.f;
    float qw = 1.f, qx = 0.f, qy = 0.f, qz = 0.f, logit = 0.f;
    if (active) {
        mx = a.means[i]; my = a.means[n + i]; mz = a.means[2 * n + i];
        ls0 = a.log_scales[i]; ls1 = a.log_scales[n + i]; ls2 = a.log_scales[2 * n + i];
        qw = a.quats[i]; qx = a.quats[n + i]; qy = a.quats[2 * n + i]; qz = a.quats[3 * n + i];
        logit = a.logits[i];
    }
    const float s0 = __expf(ls0), s1 = __expf(ls1), s2 = __expf(ls2);
    const float qn2 = qw * qw + qx * qx + qy * qy + qz * qz;
    const float qinv = rsqrtf(qn2);
    const float uw = qw * qinv, ux = qx * qinv, uy = qy * qinv, uz = qz * qinv;
    float Sg[3][3];
    {
        float Rq[9];
        quat_to_rot(uw, ux, uy, uz, Rq);
        const float M[9] = {Rq[0] * s0, Rq[1] * s1, Rq[2] * s2, Rq[3] * s0, Rq[4] * s1, Rq[5] * s2,
                            Rq[6] * s0, Rq[7] * s1, Rq[8] * s2};
        for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 3; ++c)
                Sg[r][c] = M[3 * r] * M[3 * c] + M[3 * r + 1] * M[3 * c + 1] + M[3 * r + 2] * M[3 * c + 2];
    }

    const float o = 1.f / (1.f + __expf(-logit));
    float GSig[3][3] = {{0.f, 0.f, 0.f}, {0.f, 0.f, 0.f}, {0.f, 0.f, 0.f}};
    float gmu[3] = {0.f, 0.f, 0.f};
    float go = 0.f;
    uint32_t vmask = 0;  // views keeping this Gaussian, for the colour phase
    float stat_g = 0.f, stat_c = 0.f;  // densification statistic (|dL/d(u, v)| per view)

    for (int b = 0; b < vt.n_views; ++b) {
        const bool in_range = active && i >= vt.g_begin[b] && i < vt.g_end[b];
        const long long q = vt.pair_base[b] + (i - vt.g_begin[b]);
        const bool vis = in_range && a.pair_count[q] != 0u;
        vmask |= vis ? 1u << b : 0u;
        float pose[16];
#pragma unroll
        for (int k = 0; k < 16; ++k) pose[k] = 0.f;
        if (vis) {
            const float* g2 = opaque_ptr(a.grad2d) + q * kGrad2dStride;
            // slots 0..4 hold pixel moments of dL/dpower = o h (h = dL/do per pixel) without
            // the factor o: sum h dx, h dy, h dx^2, h dx dy, h dy^2 (dx, dy = centre - pixel)
            const float M1 = o * g2[0], M2 = o * g2[1], M3 = o * g2[2], M4 = o * g2[3], M5 = o * g2[4];
            const float g_o = g2[5], g_zd = g2[9];
            const ags_camera cam = opaque_ptr(a.cams)[b];
            const float* R = cam.R;
            float x, y, z;
            world_to_cam(cam, mx, my, mz, x, y, z);
            const float rz = 1.f / z, rz2 = rz * rz;
            const float limx = a.st.fov_clamp * (float)vt.width[b] / (2.f * cam.fx);
            const float limy = a.st.fov_clamp * (float)vt.height[b] / (2.f * cam.fy);
            const float xz = x * rz, yz = y * rz;
            const bool clx = xz < -limx || xz > limx;
            const bool cly = yz < -limy || yz > limy;
            const float txz = fminf(fmaxf(xz, -limx), limx);
            const float tyz = fminf(fmaxf(yz, -limy), limy);
            const float j00 = cam.fx * rz, j02 = -cam.fx * txz * rz;
            const float j11 = cam.fy * rz, j12 = -cam.fy * tyz * rz;
            float T[2][3];
            for (int k = 0; k < 3; ++k) {
                T[0][k] = j00 * R[k] + j02 * R[6 + k];
                T[1][k] = j11 * R[3 + k] + j12 * R[6 + k];
            }
            // Sigma' = T Sigma T^T + blur
            float TS[2][3];
            for (int r = 0; r < 2; ++r)
                for (int c = 0; c < 3; ++c)
                    TS[r][c] = T[r][0] * Sg[0][c] + T[r][1] * Sg[1][c] + T[r][2] * Sg[2][c];
            const float ca = TS[0][0] * T[0][0] + TS[0][1] * T[0][1] + TS[0][2] * T[0][2] + a.st.blur;
            const float cb = TS[0][0] * T[1][0] + TS[0][1] * T[1][1] + TS[0][2] * T[1][2];
            const float cc = TS[1][0] * T[1][0] + TS[1][1] * T[1][1] + TS[1][2] * T[1][2] + a.st.blur;
            const float idet = 1.f / (ca * cc - cb * cb);
            const float KA = cc * idet, KB = -cb * idet, KC = ca * idet;
            // power = -(a dx^2 + 2 b dx dy + c dy^2) / 2 with conic (a, b, c) = (KA, KB, KC)
            const float g_u = -(KA * M1 + KB * M2), g_v = -(KB * M1 + KC * M2);
            stat_g += sqrtf(g_u * g_u + g_v * g_v);
            stat_c += 1.f;
            const float g_a = -0.5f * M3, g_b = -M4, g_c = -0.5f * M5;
            // G' = -K G_K K
            const float p = g_a, r2 = 0.5f * g_b, s = g_c;
            const float k00 = KA * p + KB * r2, k01 = KA * r2 + KB * s;
            const float k10 = KB * p + KC * r2, k11 = KB * r2 + KC * s;
            const float G00 = -(k00 * KA + k01 * KB);
            const float G01 = -(k00 * KB + k01 * KC);
            const float G11 = -(k10 * KB + k11 * KC);
            // U = G' T (2x3)
            float U[2][3];
            for (int c = 0; c < 3; ++c) {
                U[0][c] = G00 * T[0][c] + G01 * T[1][c];
                U[1][c] = G01 * T[0][c] + G11 * T[1][c];
            }
            for (int r = 0; r < 3; ++r)
                for (int c = 0; c < 3; ++c) GSig[r][c] += T[0][r] * U[0][c] + T[1][r] * U[1][c];
            // G_T = 2 U Sigma
            float GT[2][3];
            for (int r = 0; r < 2; ++r)
                for (int c = 0; c < 3; ++c)
                    GT[r][c] = 2.f * (U[r][0] * Sg[0][c] + U[r][1] * Sg[1][c] + U[r][2] * Sg[2][c]);
            // G_J = G_T R^T (only the entries of J that are not structurally zero matter)
            float GJ[2][3];
            for (int r = 0; r < 2; ++r)
                for (int m = 0; m < 3; ++m)
                    GJ[r][m] = GT[r][0] * R[3 * m] + GT[r][1] * R[3 * m + 1] + GT[r][2] * R[3 * m + 2];
            // rotation of the view through T: N = R G_T^T J, N[m][c] = sum_r GJ[r][m] J[r][c]
            // J = [[j00, 0, j02], [0, j11, j12]]
            const float N01 = GJ[1][0] * j11;
            const float N10 = GJ[0][1] * j00;
            const float N02 = GJ[0][0] * j02 + GJ[1][0] * j12;
            const float N20 = GJ[0][2] * j00;
            const float N12 = GJ[0][1] * j02 + GJ[1][1] * j12;
            const float N21 = GJ[1][2] * j11;
            // x_c adjoint
            float gx = g_u * cam.fx * rz;
            float gy = g_v * cam.fy * rz;
            float gz = -(g_u * cam.fx * x + g_v * cam.fy * y) * rz2 + g_zd;
            gz += -cam.fx * rz2 * GJ[0][0] - cam.fy * rz2 * GJ[1][1];
            if (!clx) {
                gx += -cam.fx * rz2 * GJ[0][2];
                gz += 2.f * cam.fx * x * rz2 * rz * GJ[0][2];
            } else {
                gz += cam.fx * txz * rz2 * GJ[0][2];
            }
            if (!cly) {
                gy += -cam.fy * rz2 * GJ[1][2];
                gz += 2.f * cam.fy * y * rz2 * rz * GJ[1][2];
            } else {
                gz += cam.fy * tyz * rz2 * GJ[1][2];
            }
            // mean
            gmu[0] += R[0] * gx + R[3] * gy + R[6] * gz;
            gmu[1] += R[1] * gx + R[4] * gy + R[7] * gz;
            gmu[2] += R[2] * gx + R[5] * gy + R[8] * gz;
            go += g_o;
            // pose
            pose[0] = gx;
            pose[1] = gy;
            pose[2] = gz;
            pose[3] = (y * gz - z * gy) + (N12 - N21);
            pose[4] = (z * gx - x * gz) + (N20 - N02);
            pose[5] = (x * gy - y * gx) + (N01 - N10);
        }
        if (__ballot(vis) != 0ull) {
            const float tot = wave_transpose_sum16(pose);
            const int slot = (lane >> 2) & 15;
            if ((lane & 3) == 0 && slot < 6) spose[b][slot][wave] = tot;
        }
    }
    __syncthreads();
    for (int t = threadIdx.x; t < vt.n_views * 6; t += 256) {
        const int b = t / 6, k = t % 6;
        a.pose_partials[(long long)(b * 6 + k) * (2 * gridDim.x) + blockIdx.x] =
            spose[b][k][0] + spose[b][k][1] + spose[b][k][2] + spose[b][k][3];
    }
    if (!active) return;
    a.vis_mask[i] = vmask;
    if (a.stat_grad) {
        a.stat_grad[i] += stat_g;
        a.stat_count[i] += stat_c;
    }

    // Sigma = M M^T, M = Rq diag(s): G_M = 2 G_Sigma M (G_Sigma symmetrised)
    float Rq[9];
    quat_to_rot(uw, ux, uy, uz, Rq);
    const float M[9] = {Rq[0] * s0, Rq[1] * s1, Rq[2] * s2, Rq[3] * s0, Rq[4] * s1, Rq[5] * s2,
                        Rq[6] * s0, Rq[7] * s1, Rq[8] * s2};
    float GS[3][3];
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) GS[r][c] = 0.5f * (GSig[r][c] + GSig[c][r]);
    float GM[9];
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c)
            GM[3 * r + c] = 2.f * (GS[r][0] * M[c] + GS[r][1] * M[3 + c] + GS[r][2] * M[6 + c]);
    const float sc[3] = {s0, s1, s2};
    float gls[3];
    float GR[9];
    for (int c = 0; c < 3; ++c) {
        const float gS = Rq[c] * GM[c] + Rq[3 + c] * GM[3 + c] + Rq[6 + c] * GM[6 + c];
        gls[c] = gS * sc[c];
        GR[c] = GM[c] * sc[c];
        GR[3 + c] = GM[3 + c] * sc[c];
        GR[6 + c] = GM[6 + c] * sc[c];
    }
    // rotation matrix of the unit quaternion (w, x, y, z) -> its adjoint
    const float gw = 2.f * (-uz * GR[1] + uy * GR[2] + uz * GR[3] - ux * GR[5] - uy * GR[6] + ux * GR[7]);
    const float gx_ = 2.f * (uy * GR[1] + uz * GR[2] + uy * GR[3] - uw * GR[5] + uz * GR[6] + uw * GR[7]) -
                      4.f * ux * (GR[4] + GR[8]);
    const float gy_ = 2.f * (ux * GR[1] + uw * GR[2] + ux * GR[3] + uz * GR[5] - uw * GR[6] + uz * GR[7]) -
                      4.f * uy * (GR[0] + GR[8]);
    const float gz_ = 2.f * (-uw * GR[1] + ux * GR[2] + uw * GR[3] + uy * GR[5] + ux * GR[6] + uy * GR[7]) -
                      4.f * uz * (GR[0] + GR[4]);
    // normalisation q / |q|
    const float dot = uw * gw + ux * gx_ + uy * gy_ + uz * gz_;
    const float gq[4] = {(gw - uw * dot) * qinv, (gx_ - ux * dot) * qinv, (gy_ - uy * dot) * qinv,
                         (gz_ - uz * dot) * qinv};
    const float glogit = go * o * (1.f - o);

    if (a.accumulate) {
        for (int c = 0; c < 3; ++c) {
            a.g_means[c * n + i] += gmu[c];
            a.g_log_scales[c * n + i] += gls[c];
        }
        for (int c = 0; c < 4; ++c) a.g_quats[c * n + i] += gq[c];
        a.g_logits[i] += glogit;
    } else {
        for (int c = 0; c < 3; ++c) {
            a.g_means[c * n + i] = gmu[c];
            a.g_log_scales[c * n + i] = gls[c];
        }
        for (int c = 0; c < 4; ++c) a.g_quats[c * n + i] = gq[c];
        a.g_logits[i] = glogit;
    }
}

// Colour adjoint through the SH evaluation: dL/df_kc = sum over the views keeping the
// Gaussian of Y_k(d_b) gcol_b,c, with gcol the colour adjoint of the pair masked where the
// forward clamped the colour at 0 (stored colour == 0); and the direction term
// g_dir = P_d (sum_c gcol_c sum_k f_kc grad Y_k(d)) / |mu - C_b| (P_d the projection on the
// tangent plane of the unit sphere), added to dL/dmu and, as R_b g_dir, to the view's
// dL/drho.  One thread per Gaussian; its K x 3 coefficients are read once, the K x 3 sums
// stay in registers and are written once (or, with FUSED, applied by Adam at once).
template <int DEG, bool FUSED>
__device__ __forceinline__ void colour_bwd(const ProjectBwdArgs& a) {
    constexpr int K = (DEG + 1) * (DEG + 1);
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const bool active = i < a.n;
    const int n = a.n;
    const int lane = __lane_id(), wave = threadIdx.x >> 6;
    const ViewTable& vt = a.vt;
    __shared__ float spose[kMaxViews][3][4];
    // second half of each partials row (the geometry phase fills the first)
    float* partials = a.pose_partials + gridDim.x;

    float mx = 0.f, my = 0.f, mz = 0.f;
    uint32_t vis = 0;
    if (active) {
        mx = a.means[i]; my = a.means[n + i]; mz = a.means[2 * n + i];
        vis = a.vis_mask[i];
    }
    float f[K][3];
    if (DEG > 0 && vis) {
#pragma unroll
        for (int k = 0; k < K; ++k)
#pragma unroll
            for (int c = 0; c < 3; ++c) f[k][c] = sh_row(a.sh, n, k * 3 + c)[(uint32_t)i];
    }
    float acc[K][3];
#pragma unroll
    for (int k = 0; k < K; ++k) acc[k][0] = acc[k][1] = acc[k][2] = 0.f;
    float gm[3] = {0.f, 0.f, 0.f};
    for (int b = 0; b < vt.n_views; ++b) {
        const bool on = (vis >> b) & 1u;
        float pr[3] = {0.f, 0.f, 0.f};
        if (on) {
            const long long q = vt.pair_base[b] + (i - vt.g_begin[b]);
            // both reads issued together (vector loads), then the mask
            const float4 rc = reinterpret_cast<const float4*>(a.records + q * kRecFloats)[2];  // ey, r, g, b
            const float2* g2 = reinterpret_cast<const float2*>(a.grad2d + q * kGrad2dStride);
            const float2 g67 = g2[3], g89 = g2[4];
            const float gcol[3] = {rc.y > 0.f ? g67.x : 0.f, rc.z > 0.f ? g67.y : 0.f, rc.w > 0.f ? g89.x : 0.f};
            const ags_camera cam = a.cams[b];
            const float* R = cam.R;
            float dx, dy, dz;
            centre_to_mean(cam, mx, my, mz, dx, dy, dz);
            const float il = rsqrtf(dx * dx + dy * dy + dz * dz);
            dx *= il; dy *= il; dz *= il;
            float Y[16];
            sh_basis(DEG, dx, dy, dz, Y);
#pragma unroll
            for (int k = 0; k < K; ++k) {
                acc[k][0] += Y[k] * gcol[0];
                acc[k][1] += Y[k] * gcol[1];
                acc[k][2] += Y[k] * gcol[2];
            }
            if (DEG > 0) {
                // sum_c gcol_c grad(sum_k f_kc Y_k) = grad(sum_k w_k Y_k), w_k = sum_c gcol_c f_kc
                float w[16], gdir[3];
#pragma unroll
                for (int k = 0; k < K; ++k) w[k] = gcol[0] * f[k][0] + gcol[1] * f[k][1] + gcol[2] * f[k][2];
                sh_grad_dot(DEG, dx, dy, dz, w, gdir);
                const float dd = gdir[0] * dx + gdir[1] * dy + gdir[2] * dz;
                gdir[0] = (gdir[0] - dd * dx) * il;
                gdir[1] = (gdir[1] - dd * dy) * il;
                gdir[2] = (gdir[2] - dd * dz) * il;
                gm[0] += gdir[0];
                gm[1] += gdir[1];
                gm[2] += gdir[2];
                pr[0] = R[0] * gdir[0] + R[1] * gdir[1] + R[2] * gdir[2];
                pr[1] = R[3] * gdir[0] + R[4] * gdir[1] + R[5] * gdir[2];
                pr[2] = R[6] * gdir[0] + R[7] * gdir[1] + R[8] * gdir[2];
            }
        }
        if (DEG > 0) {
            float s0 = 0.f, s1 = 0.f, s2 = 0.f;
            if (__ballot(on) != 0ull) {
                s0 = wave_sum(pr[0]);
                s1 = wave_sum(pr[1]);
                s2 = wave_sum(pr[2]);
            }
            if (lane == 0) {
                spose[b][0][wave] = s0;
                spose[b][1][wave] = s1;
                spose[b][2][wave] = s2;
            }
        }
    }
    __syncthreads();
    for (int t = threadIdx.x; t < vt.n_views * 6; t += 256) {
        const int b = t / 6, k = t % 6;
        partials[(long long)(b * 6 + k) * (2 * gridDim.x) + blockIdx.x] =
            (DEG > 0 && k < 3) ? spose[b][k][0] + spose[b][k][1] + spose[b][k][2] + spose[b][k][3] : 0.f;
    }
    if (!active) return;
    if (FUSED) {
        // the Gaussian's gradient is complete here: update all its parameters in place, in
        // batches whose loads are all issued before any of the batch's stores
        const AdamArgs& ad = a.adam;
        const float t = (float)(*ad.step);
        const float b1 = ad.beta1, b2 = ad.beta2, eps = ad.eps;
        const float bc1 = 1.f - powf(b1, t), bc2 = 1.f - powf(b2, t);
        constexpr int R = 3 * K, CH = 8;  // SH rows (coefficient k, channel c) = 3 k + c
#pragma unroll
        for (int r0 = 0; r0 < R; r0 += CH) {
            float pp[CH], mm[CH], vv[CH];
#pragma unroll
            for (int j = 0; j < CH; ++j)
                if (r0 + j < R) {
                    const long long e = (long long)(r0 + j) * n + i;
                    pp[j] = ad.p[4][e];
                    mm[j] = ad.m[4][e];
                    vv[j] = ad.v[4][e];
                }
#pragma unroll
            for (int j = 0; j < CH; ++j)
                if (r0 + j < R)
                    adam_one(pp[j], acc[(r0 + j) / 3][(r0 + j) % 3], mm[j], vv[j], r0 + j < 3 ? ad.lr[4] : ad.lr[5], b1,
                             b2, bc1, bc2, eps);
#pragma unroll
            for (int j = 0; j < CH; ++j)
                if (r0 + j < R) {
                    const long long e = (long long)(r0 + j) * n + i;
                    ad.p[4][e] = pp[j];
                    ad.m[4][e] = mm[j];
                    ad.v[4][e] = vv[j];
                }
        }
        // means (with the direction term), log-scales, quaternion, logit: 11 rows
        float* const P[11] = {ad.p[0], ad.p[0] + n, ad.p[0] + 2 * (long long)n, ad.p[1], ad.p[1] + n,
                              ad.p[1] + 2 * (long long)n, ad.p[2], ad.p[2] + n, ad.p[2] + 2 * (long long)n,
                              ad.p[2] + 3 * (long long)n, ad.p[3]};
        float* const Mo[11] = {ad.m[0], ad.m[0] + n, ad.m[0] + 2 * (long long)n, ad.m[1], ad.m[1] + n,
                               ad.m[1] + 2 * (long long)n, ad.m[2], ad.m[2] + n, ad.m[2] + 2 * (long long)n,
                               ad.m[2] + 3 * (long long)n, ad.m[3]};
        float* const Vo[11] = {ad.v[0], ad.v[0] + n, ad.v[0] + 2 * (long long)n, ad.v[1], ad.v[1] + n,
                               ad.v[1] + 2 * (long long)n, ad.v[2], ad.v[2] + n, ad.v[2] + 2 * (long long)n,
                               ad.v[2] + 3 * (long long)n, ad.v[3]};
        const float* const G[11] = {a.g_means, a.g_means + n, a.g_means + 2 * (long long)n, a.g_log_scales,
                                    a.g_log_scales + n, a.g_log_scales + 2 * (long long)n, a.g_quats,
                                    a.g_quats + n, a.g_quats + 2 * (long long)n, a.g_quats + 3 * (long long)n,
                                    a.g_logits};
        float pp[11], mm[11], vv[11], gg[11];
#pragma unroll
        for (int j = 0; j < 11; ++j) {
            pp[j] = P[j][i];
            mm[j] = Mo[j][i];
            vv[j] = Vo[j][i];
            gg[j] = G[j][i];
        }
#pragma unroll
        for (int j = 0; j < 3; ++j) gg[j] = gg[j] + gm[j];
#pragma unroll
        for (int j = 0; j < 11; ++j) {
            const float lr = j < 3 ? ad.lr[0] : j < 6 ? ad.lr[1] : j < 10 ? ad.lr[2] : ad.lr[3];
            adam_one(pp[j], gg[j], mm[j], vv[j], lr, b1, b2, bc1, bc2, eps);
        }
#pragma unroll
        for (int j = 0; j < 11; ++j) {
            P[j][i] = pp[j];
            Mo[j][i] = mm[j];
            Vo[j][i] = vv[j];
        }
        return;
    }
    if (a.accumulate) {
#pragma unroll
        for (int k = 0; k < K; ++k)
#pragma unroll
            for (int c = 0; c < 3; ++c) sh_row(a.g_sh, n, k * 3 + c)[(uint32_t)i] += acc[k][c];
    } else {
        // plain stores (no read of the old values)
#pragma unroll
        for (int k = 0; k < K; ++k)
#pragma unroll
            for (int c = 0; c < 3; ++c) sh_row(a.g_sh, n, k * 3 + c)[(uint32_t)i] = acc[k][c];
    }
    if (DEG > 0) {
        a.g_means[i] += gm[0];
        a.g_means[n + i] += gm[1];
        a.g_means[2 * n + i] += gm[2];
    }
}

// Both phases for one Gaussian per thread: the geometry adjoint, then the colour adjoint
// (with FUSED, followed by the Adam step on all of the Gaussian's parameters).
template <int DEG, bool FUSED>
__global__ __launch_bounds__(256) void project_bwd_kernel(ProjectBwdArgs a) {
    geometry_bwd<DEG>(a);
    colour_bwd<DEG, FUSED>(a);
}

// Sum of the per-workgroup pose partials, fixed order: one workgroup per (view, component),
// whose partials form one contiguous row of n_blocks values; with loss_out, one more
// workgroup adds up the loss partials (fixed order, the skipped range counting as zero).
__global__ __launch_bounds__(256) void pose_reduce_kernel(const float* partials, int n_blocks, int n_views,
                                                         float* pose, int accumulate, const float* lp, long long n_lp,
                                                         long long skip0, long long skip1, float* loss_out) {
    __shared__ float sred[4];
    const int bk = blockIdx.x;  // b * 6 + k
    if (bk == n_views * 6) {
        float acc[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        auto at = [&](long long j) { return j >= skip0 && j < skip1 ? 0.f : lp[j]; };
        long long i = threadIdx.x;
        for (; i + 7 * 256 < n_lp; i += 8 * 256)
#pragma unroll
            for (int u = 0; u < 8; ++u) acc[u] += at(i + u * 256);
#pragma unroll
        for (int u = 0; u < 8; ++u)
            if (i + u * 256 < n_lp) acc[u] += at(i + u * 256);
        float s = ((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7]));
        s = wave_sum(s);
        if ((threadIdx.x & 63) == 0) sred[threadIdx.x >> 6] = s;
        __syncthreads();
        if (threadIdx.x == 0) loss_out[0] = (sred[0] + sred[1]) + (sred[2] + sred[3]);
        return;
    }
    const float* row = partials + (long long)bk * n_blocks;
    float s0 = 0.f, s1 = 0.f, s2 = 0.f, s3 = 0.f;
    int g = threadIdx.x;
    for (; g + 768 < n_blocks; g += 1024) {
        s0 += row[g];
        s1 += row[g + 256];
        s2 += row[g + 512];
        s3 += row[g + 768];
    }
    for (; g < n_blocks; g += 256) s0 += row[g];
    float s = (s0 + s1) + (s2 + s3);
    (void)n_views;
    s = wave_sum(s);
    if ((threadIdx.x & 63) == 0) sred[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        const float t = sred[0] + sred[1] + sred[2] + sred[3];
        pose[bk] = accumulate ? pose[bk] + t : t;
    }
}

int project_bwd_blocks(int n) { return n > 0 ? (n + 255) / 256 : 0; }

void launch_project_bwd(const ProjectBwdArgs& a, hipStream_t s) {
    const int nb = project_bwd_blocks(a.n);
    if (nb > 0) launch_project_bwd_main(a, s);
    if (nb > 0) {
        hipLaunchKernelGGL(pose_reduce_kernel, dim3(a.vt.n_views * 6 + (a.loss_out ? 1 : 0)), dim3(256), 0, s,
                           a.pose_partials, 2 * nb, a.vt.n_views, a.g_pose, a.accumulate, a.loss_partials, a.n_loss,
                           a.loss_skip0, a.loss_skip1, a.loss_out);
        return;
    }
    if (!a.accumulate) launch_fill_f32(a.g_pose, 0.f, 6LL * a.vt.n_views, s);
    if (a.loss_out) launch_sum_partials(a.loss_partials, a.n_loss, a.loss_skip0, a.loss_skip1, a.loss_out, s);
}

void launch_project_bwd_main(const ProjectBwdArgs& a, hipStream_t s) {
    dim3 grid((a.n + 255) / 256), block(256);
#define PB(d_)                                                                                 \
    do {                                                                                       \
        if (a.fused_adam)                                                                      \
            hipLaunchKernelGGL((project_bwd_kernel<d_, true>), grid, block, 0, s, a);           \
        else                                                                                   \
            hipLaunchKernelGGL((project_bwd_kernel<d_, false>), grid, block, 0, s, a);          \
    } while (0)
    switch (a.sh_degree) {
        case 0: PB(0); break;
        case 1: PB(1); break;
        case 2: PB(2); break;
        default: PB(3); break;
    }
#undef PB
}

}  // namespace ags
