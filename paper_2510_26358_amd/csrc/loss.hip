// LiDAR depth-consistency adjoint (Sec. III-C, probabilistic depth term).
//
// Each LiDAR return j of view b at pixel p_j is N(D_j, s_j^2); the renderer's depth
// distribution there is N(mu, v) with mu the composited expected depth and
//   v = s_j^2 (fixed-variance reading: the term is (mu - D_j)^2 / (2 s_j^2), adjoint
//       (mu - D_j) / s_j^2), or
//   v = M2 - mu^2 + floor, M2 = sum w z^2 (rendered variance, from the forward's variance
//       output): with e = D_j - mu and
//       K = KL(N(D_j, s^2) || N(mu, v)) = ln(sqrt(v) / s) + (s^2 + e^2) / (2 v) - 1/2,
//       dK/dv = 1 / (2 v) - (s^2 + e^2) / (2 v^2), dK/dM2 = dK/dv, dK/dmu = -e / v - 2 mu dK/dv.
// Each term is scaled by lambda / |Omega_b|; the adjoints go into dense per-pixel buffers
// (depth, and second moment) that the raster backward reads.
#include "common.h"

namespace ags {

constexpr int kLidarThreads = 256;
constexpr int kLidarBlocks = 256;  // fixed grid: the loss partials buffer has one slot per block

int lidar_blocks(long long) { return kLidarBlocks; }

__global__ __launch_bounds__(kLidarThreads) void lidar_adjoint_kernel(LidarArgs a) {
    __shared__ float sred[kLidarThreads / 64];
    float part = 0.f;
    for (long long j = (long long)blockIdx.x * kLidarThreads + threadIdx.x; j < a.n_targets;
         j += (long long)kLidarBlocks * kLidarThreads) {
        int b = 0;
        for (int k = 1; k < a.vt.n_views; ++k)
            if (j >= a.target_off[k]) b = k;
        const int pj = a.pix[j];
        if (pj < 0 || (long long)pj >= (long long)a.vt.width[b] * a.vt.height[b]) {
            // a target outside its view: no adjoint, and the loss becomes NaN so that the
            // caller sees the bad input (the host cannot read device targets without a sync)
            part = __builtin_nanf("");
            continue;
        }
        const long long gp = a.vt.pix_base[b] + pj;
        const float mu = a.depth[gp];
        const float s = a.sigma[j];
        const float r = mu - a.val[j];
        if (a.depth_var) {
            const float v = a.depth_var[gp] + a.sigma_floor;
            const float iv = 1.f / v;
            const float q = s * s + r * r;
            const float dv = 0.5f * iv - 0.5f * q * iv * iv;
            atomicAdd(a.d_depth + gp, a.scale[b] * (r * iv - 2.f * mu * dv));
            atomicAdd(a.d_depth2 + gp, a.scale[b] * dv);
            part += a.scale[b] * (0.5f * __logf(v / (s * s)) + 0.5f * q * iv - 0.5f);
        } else {
            const float is2 = 1.f / (s * s);
            atomicAdd(a.d_depth + gp, a.scale[b] * r * is2);
            part += a.scale[b] * 0.5f * r * r * is2;
        }
    }
    part = wave_sum(part);
    if ((threadIdx.x & 63) == 0) sred[threadIdx.x >> 6] = part;
    __syncthreads();
    if (threadIdx.x == 0) {
        float s = 0.f;
        for (int w = 0; w < kLidarThreads / 64; ++w) s += sred[w];
        a.loss_partials[blockIdx.x] = s;
    }
}

void launch_lidar_adjoint(const LidarArgs& a, hipStream_t s) {
    hipLaunchKernelGGL(lidar_adjoint_kernel, dim3(kLidarBlocks), dim3(kLidarThreads), 0, s, a);
}

// Deterministic sum of the per-block loss partials (fixed order, one workgroup); the entries
// in [skip0, skip1) belong to terms that are off, were not written, and count as zero.
__global__ __launch_bounds__(1024) void sum_partials_kernel(const float* p, long long n, long long skip0,
                                                            long long skip1, float* out) {
    __shared__ float sred[16];
    // eight independent sums per thread, so eight loads are in flight at a time (fixed order)
    float acc[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    long long i = threadIdx.x;
    auto at = [&](long long j) { return j >= skip0 && j < skip1 ? 0.f : p[j]; };
    for (; i + 7 * 1024 < n; i += 8 * 1024)
#pragma unroll
        for (int u = 0; u < 8; ++u) acc[u] += at(i + u * 1024);
#pragma unroll
    for (int u = 0; u < 8; ++u)
        if (i + u * 1024 < n) acc[u] += at(i + u * 1024);
    float s = ((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7]));
    s = wave_sum(s);
    if ((threadIdx.x & 63) == 0) sred[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        float t = 0.f;
        for (int w = 0; w < 16; ++w) t += sred[w];
        out[0] = t;
    }
}

void launch_sum_partials(const float* partials, long long n, long long skip0, long long skip1, float* out,
                         hipStream_t s) {
    hipLaunchKernelGGL(sum_partials_kernel, dim3(1), dim3(1024), 0, s, partials, n, skip0, skip1, out);
}

}  // namespace ags
