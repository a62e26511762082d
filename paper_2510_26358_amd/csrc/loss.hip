// LiDAR depth-consistency adjoint (Sec. III-C, probabilistic depth term).
//
// Each LiDAR return j of view b at pixel p_j is N(D_j, s_j^2); the renderer's depth
// distribution there is N(mu, s_j^2) with mu the composited expected depth (fixed
// variance reading, sigma_u = sigma_L).  The term lambda / |Omega_b| KL(.||.) equals
// lambda / |Omega_b| (mu - D_j)^2 / (2 s_j^2); its adjoint lambda / |Omega_b| (mu - D_j) / s_j^2
// is added into a dense per-pixel depth adjoint that the raster backward reads.
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
        if (pj < 0 || (long long)pj >= (long long)a.vt.width[b] * a.vt.height[b]) continue;
        const long long gp = a.vt.pix_base[b] + pj;
        const float mu = a.depth[gp];
        const float s = a.sigma[j];
        const float r = mu - a.val[j];
        const float is2 = 1.f / (s * s);
        atomicAdd(a.d_depth + gp, a.scale[b] * r * is2);
        part += a.scale[b] * 0.5f * r * r * is2;
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

// Deterministic sum of the per-block loss partials (fixed order, one workgroup).
__global__ __launch_bounds__(1024) void sum_partials_kernel(const float* p, long long n, float* out) {
    __shared__ float sred[16];
    float s = 0.f;
    for (long long i = threadIdx.x; i < n; i += 1024) s += p[i];
    s = wave_sum(s);
    if ((threadIdx.x & 63) == 0) sred[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        float t = 0.f;
        for (int w = 0; w < 16; ++w) t += sred[w];
        out[0] = t;
    }
}

void launch_sum_partials(const float* partials, long long n, float* out, hipStream_t s) {
    hipLaunchKernelGGL(sum_partials_kernel, dim3(1), dim3(1024), 0, s, partials, n, out);
}

}  // namespace ags
