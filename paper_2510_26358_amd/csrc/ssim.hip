// D-SSIM part of the photometric loss (Sec. III-C: L_3DGS = (1 - lambda) L1 + lambda D-SSIM)
// and its adjoint with respect to the rendered colour, for all views in one launch.
//
// Per pixel p and channel: with G the 11 x 11 Gaussian window (sigma 1.5, weights summing to
// 1, zero padding), mu_x = G * x, E_xx = G * x^2, E_xy = G * (x y) (y = target),
//   A1 = 2 mu_x mu_y + C1,  A2 = 2 (E_xy - mu_x mu_y) + C2,
//   B1 = mu_x^2 + mu_y^2 + C1,  B2 = (E_xx - mu_x^2) + (E_yy - mu_y^2) + C2,  s = A1 A2 / (B1 B2).
// The loss adds sum_p m_p (1 - s_p) per channel, m_p = lambda w_l1 / (3 n_b) on the pixels of
// the L1 mask (all pixels without one).  Its adjoint: with the partial derivatives of s at
// fixed window moments
//   D_mu = 2 mu_y (A2 - A1) / (B1 B2) + 2 mu_x s (1 / B2 - 1 / B1),
//   D_xx = -s / B2,   D_xy = 2 A1 / (B1 B2),
// dL/dx_q = -[G * (m D_mu)](q) - 2 x_q [G * (m D_xx)](q) - y_q [G * (m D_xy)](q)
// (the window is symmetric, so the transposed blur is the blur).
//
// One workgroup per 32 x 32 output tile and colour channel: the inputs with a 10-pixel halo
// go to LDS, the five window moments are blurred over the tile plus a 5-pixel halo
// (row pass, then column pass), D is formed there, blurred back onto the tile and combined
// with x and y.  Each thread runs a blur over a short segment of one row or column with the
// segment's inputs in registers, so every LDS value read feeds several outputs.
#include "common.h"

namespace ags {

constexpr int kSsimTO = 32;                     // output tile edge
constexpr int kSsimR = 5;                       // window radius
constexpr int kSsimIn = kSsimTO + 4 * kSsimR;   // 52: inputs with the double halo
constexpr int kSsimMid = kSsimTO + 2 * kSsimR;  // 42: moments / D with the single halo
constexpr int kSsimThreads = 512;
constexpr float kSsimC1 = 0.01f * 0.01f;
constexpr float kSsimC2 = 0.03f * 0.03f;

int ssim_tiles(const ViewTable& vt, int b) {
    return ((vt.width[b] + kSsimTO - 1) / kSsimTO) * ((vt.height[b] + kSsimTO - 1) / kSsimTO);
}

long long ssim_blocks(const ViewTable& vt) {
    long long t = 0;
    for (int b = 0; b < vt.n_views; ++b) t += ssim_tiles(vt, b);
    return 3 * t;
}

// LDS: the inputs (steps 1-2) share their space with D (steps 3-4), which is why step 5
// reads x and y of the tile again from global memory (cache hits); 65 KB lets two
// workgroups share a CU.
union SsimFront {
    struct {
        float x[kSsimIn][kSsimIn], y[kSsimIn][kSsimIn];
    } in;
    float d[3][kSsimMid][kSsimMid];
};

__global__ __launch_bounds__(kSsimThreads) void ssim_kernel(SsimArgs a) {
    __shared__ SsimFront front;
    __shared__ float hbuf[5][kSsimIn][kSsimMid];  // row-blurred moments; later the row-blurred D
    __shared__ float sred[kSsimThreads / 64];
    auto& sX = front.in.x;
    auto& sY = front.in.y;
    auto& sD = front.d;
    const ViewTable& vt = a.vt;
    const int tid = threadIdx.x;
    const int c = blockIdx.y;  // colour channel
    // view and tile of this workgroup
    int b = 0, t = blockIdx.x;
    while (b + 1 < vt.n_views && t >= a.tile_base[b + 1]) ++b;
    t -= a.tile_base[b];
    const int W = vt.width[b], H = vt.height[b];
    const int ntx = (W + kSsimTO - 1) / kSsimTO;
    const int ox = (t % ntx) * kSsimTO, oy = (t / ntx) * kSsimTO;
    const long long plane = (long long)W * H;
    const float* X = a.rgb + 3 * vt.pix_base[b] + c * plane;
    const float* Y = a.gt_rgb + 3 * vt.pix_base[b] + c * plane;
    float w[2 * kSsimR + 1];
#pragma unroll
    for (int k = 0; k < 2 * kSsimR + 1; ++k) w[k] = a.w[k];

    // 1. inputs over [ox - 2R, ox + TO + 2R)^2, zero outside the image; all loads issued
    //    before the first store
    {
        constexpr int kN = (kSsimIn * kSsimIn + kSsimThreads - 1) / kSsimThreads;
        float vx[kN], vy[kN];
#pragma unroll
        for (int j = 0; j < kN; ++j) {
            const int i = tid + j * kSsimThreads;
            const int r = i / kSsimIn, q = i % kSsimIn;
            const int y = oy - 2 * kSsimR + r, x = ox - 2 * kSsimR + q;
            const bool in = i < kSsimIn * kSsimIn && x >= 0 && x < W && y >= 0 && y < H;
            const long long p = (long long)y * W + x;
            vx[j] = in ? X[p] : 0.f;
            vy[j] = in ? Y[p] : 0.f;
        }
#pragma unroll
        for (int j = 0; j < kN; ++j) {
            const int i = tid + j * kSsimThreads;
            if (i < kSsimIn * kSsimIn) {
                sX[i / kSsimIn][i % kSsimIn] = vx[j];
                sY[i / kSsimIn][i % kSsimIn] = vy[j];
            }
        }
    }
    __syncthreads();

    // 2. row pass of x, y, x^2, y^2, x y: all 52 rows, the 42 middle columns, 7 outputs per item
    for (int it = tid; it < kSsimIn * 6; it += kSsimThreads) {
        const int r = it / 6, c0 = (it % 6) * 7;
        float xs[17], ys[17];
#pragma unroll
        for (int k = 0; k < 17; ++k) {
            xs[k] = sX[r][c0 + k];
            ys[k] = sY[r][c0 + k];
        }
#pragma unroll
        for (int o = 0; o < 7; ++o) {
            float m0 = 0.f, m1 = 0.f, m2 = 0.f, m3 = 0.f, m4 = 0.f;
#pragma unroll
            for (int k = 0; k < 2 * kSsimR + 1; ++k) {
                const float u = xs[o + k], v = ys[o + k];
                m0 += w[k] * u;
                m1 += w[k] * v;
                m2 += w[k] * (u * u);
                m3 += w[k] * (v * v);
                m4 += w[k] * (u * v);
            }
            hbuf[0][r][c0 + o] = m0;
            hbuf[1][r][c0 + o] = m1;
            hbuf[2][r][c0 + o] = m2;
            hbuf[3][r][c0 + o] = m3;
            hbuf[4][r][c0 + o] = m4;
        }
    }
    __syncthreads();

    // 3. column pass -> moments over the 42 x 42 middle region; s, D and the loss there
    const float mscale = a.scale[b];
    float part = 0.f;
    for (int it = tid; it < kSsimMid * 6; it += kSsimThreads) {
        const int q = it % kSsimMid, r0 = (it / kSsimMid) * 7;
        float mom[5][7];
#pragma unroll
        for (int m = 0; m < 5; ++m) {
            float col[17];
#pragma unroll
            for (int k = 0; k < 17; ++k) col[k] = hbuf[m][r0 + k][q];
#pragma unroll
            for (int o = 0; o < 7; ++o) {
                float acc = 0.f;
#pragma unroll
                for (int k = 0; k < 2 * kSsimR + 1; ++k) acc += w[k] * col[o + k];
                mom[m][o] = acc;
            }
        }
        const int x = ox - kSsimR + q;
#pragma unroll
        for (int o = 0; o < 7; ++o) {
            const int r = r0 + o, y = oy - kSsimR + r;
            const float mx = mom[0][o], my = mom[1][o];
            const float A1 = 2.f * mx * my + kSsimC1;
            const float A2 = 2.f * (mom[4][o] - mx * my) + kSsimC2;
            const float B1 = mx * mx + my * my + kSsimC1;
            const float B2 = (mom[2][o] - mx * mx) + (mom[3][o] - my * my) + kSsimC2;
            const float rB1 = __builtin_amdgcn_rcpf(B1), rB2 = __builtin_amdgcn_rcpf(B2);
            const float iB = rB1 * rB2;
            const float s = A1 * A2 * iB;
            bool on = x >= 0 && x < W && y >= 0 && y < H;
            if (on && a.mask) on = a.mask[vt.pix_base[b] + (long long)y * W + x] != 0;
            const float m = on ? mscale : 0.f;
            sD[0][r][q] = m * (2.f * my * (A2 - A1) * iB + 2.f * mx * s * (rB2 - rB1));
            sD[1][r][q] = m * (-s * rB2);
            sD[2][r][q] = m * (2.f * A1 * iB);
            if (r >= kSsimR && r < kSsimR + kSsimTO && q >= kSsimR && q < kSsimR + kSsimTO) part += m * (1.f - s);
        }
    }
    __syncthreads();

    // 4. row pass of m D over the 42 rows onto the 32 tile columns (into hbuf), 8 outputs per item
    //    (one map per item: 3 x 42 x 4 items)
    for (int it = tid; it < 3 * kSsimMid * 4; it += kSsimThreads) {
        const int m = it / (kSsimMid * 4), rem = it % (kSsimMid * 4);
        const int r = rem / 4, c0 = (rem % 4) * 8;
        float row[18];
#pragma unroll
        for (int k = 0; k < 18; ++k) row[k] = sD[m][r][c0 + k];
#pragma unroll
        for (int o = 0; o < 8; ++o) {
            float acc = 0.f;
#pragma unroll
            for (int k = 0; k < 2 * kSsimR + 1; ++k) acc += w[k] * row[o + k];
            hbuf[m][r][c0 + o] = acc;
        }
    }
    __syncthreads();

    // 5. column pass onto the tile; combine with x and y (read again: their LDS now holds D)
    //    (4 rows per item: 32 x 8 items)
    for (int it = tid; it < kSsimTO * 8; it += kSsimThreads) {
        const int q = it % kSsimTO, r0 = (it / kSsimTO) * 4;
        const int x = ox + q;
        float xv[4], yv[4];
#pragma unroll
        for (int o = 0; o < 4; ++o) {
            const int y = oy + r0 + o;
            const bool in = x < W && y < H;
            const long long p = (long long)y * W + x;
            xv[o] = in ? X[p] : 0.f;
            yv[o] = in ? Y[p] : 0.f;
        }
        float g[3][4];
#pragma unroll
        for (int m = 0; m < 3; ++m) {
            float col[14];
#pragma unroll
            for (int k = 0; k < 14; ++k) col[k] = hbuf[m][r0 + k][q];
#pragma unroll
            for (int o = 0; o < 4; ++o) {
                float acc = 0.f;
#pragma unroll
                for (int k = 0; k < 2 * kSsimR + 1; ++k) acc += w[k] * col[o + k];
                g[m][o] = acc;
            }
        }
#pragma unroll
        for (int o = 0; o < 4; ++o) {
            const int y = oy + r0 + o;
            if (x < W && y < H)
                a.d_rgb[3 * vt.pix_base[b] + c * plane + (long long)y * W + x] =
                    -(g[0][o] + 2.f * xv[o] * g[1][o] + yv[o] * g[2][o]);
        }
    }

    // workgroup sum of the loss part, one partial per workgroup
    part = wave_sum(part);
    if ((tid & 63) == 0) sred[tid >> 6] = part;
    __syncthreads();
    if (tid == 0) {
        float s = 0.f;
        for (int i = 0; i < kSsimThreads / 64; ++i) s += sred[i];
        a.partials[(long long)blockIdx.y * gridDim.x + blockIdx.x] = s;
    }
}

void launch_ssim(SsimArgs a, hipStream_t s) {
    int tb = 0;
    for (int b = 0; b < a.vt.n_views; ++b) {
        a.tile_base[b] = tb;
        tb += ssim_tiles(a.vt, b);
    }
    a.tile_base[a.vt.n_views] = tb;
    if (tb == 0) return;
    // the zero-mean-free Gaussian window, normalised in double
    double wd[2 * kSsimR + 1], sum = 0.0;
    for (int k = 0; k <= 2 * kSsimR; ++k) {
        const double d = k - kSsimR;
        wd[k] = std::exp(-d * d / (2.0 * 1.5 * 1.5));
        sum += wd[k];
    }
    for (int k = 0; k <= 2 * kSsimR; ++k) a.w[k] = (float)(wd[k] / sum);
    hipLaunchKernelGGL(ssim_kernel, dim3(tb, 3), dim3(kSsimThreads), 0, s, a);
}

}  // namespace ags
