// Joint refinement updates: Adam on the Gaussian parameters and Adam on each camera's
// se(3) increment followed by the left retraction W <- Exp(delta) W.  The paper refines
// splats and poses jointly by gradient steps on the multimodal loss (Sec. III-C); Adam and
// the tangent-space pose update are the refinement workload's choice.  The step number is
// read from device memory so a captured optimisation step can be replayed unchanged.
#include "common.h"

namespace ags {

// Grid row y = parameter group (means, log-scales, quaternions, logits, SH degree 0, SH
// degree >= 1), each a contiguous run of the SoA buffers; a thread updates four consecutive
// values per step with 16-byte accesses when the group's four buffers allow them.
__global__ __launch_bounds__(256) void adam_kernel(AdamArgs a) {
    const int grp = blockIdx.y;
    const long long n = a.n;
    const int seg = grp < 5 ? grp : 4;  // both SH groups live in the SH buffers
    const long long off = grp == 5 ? 3 * n : 0;
    const long long len = grp == 0 ? 3 * n : grp == 1 ? 3 * n : grp == 2 ? 4 * n : grp == 3 ? n
                        : grp == 4 ? (a.sh_k > 0 ? 3 * n : 0) : (long long)(a.sh_k - 1) * 3 * n;
    if (len <= 0) return;
    float* p = a.p[seg] + off;
    const float* g = a.g[seg] + off;
    float* m = a.m[seg] + off;
    float* v = a.v[seg] + off;
    const float lr = a.lr[grp];
    const float b1 = a.beta1, b2 = a.beta2, eps = a.eps;
    const float t = (float)(*a.step);
    const float bc1 = 1.f - powf(b1, t);
    const float bc2 = 1.f - powf(b2, t);
    const bool vec = ((reinterpret_cast<uintptr_t>(p) | reinterpret_cast<uintptr_t>(g) |
                       reinterpret_cast<uintptr_t>(m) | reinterpret_cast<uintptr_t>(v)) & 15u) == 0;
    const long long stride = 4LL * gridDim.x * blockDim.x;
    for (long long e = 4LL * ((long long)blockIdx.x * blockDim.x + threadIdx.x); e < len; e += stride) {
        if (vec && e + 4 <= len) {
            float4 pp = *reinterpret_cast<float4*>(p + e);
            const float4 gg = *reinterpret_cast<const float4*>(g + e);
            float4 mm = *reinterpret_cast<float4*>(m + e);
            float4 vv = *reinterpret_cast<float4*>(v + e);
            adam_one(pp.x, gg.x, mm.x, vv.x, lr, b1, b2, bc1, bc2, eps);
            adam_one(pp.y, gg.y, mm.y, vv.y, lr, b1, b2, bc1, bc2, eps);
            adam_one(pp.z, gg.z, mm.z, vv.z, lr, b1, b2, bc1, bc2, eps);
            adam_one(pp.w, gg.w, mm.w, vv.w, lr, b1, b2, bc1, bc2, eps);
            *reinterpret_cast<float4*>(p + e) = pp;
            *reinterpret_cast<float4*>(m + e) = mm;
            *reinterpret_cast<float4*>(v + e) = vv;
        } else {
            const long long e1 = e + 4 < len ? e + 4 : len;
            for (long long j = e; j < e1; ++j) adam_one(p[j], g[j], m[j], v[j], lr, b1, b2, bc1, bc2, eps);
        }
    }
}

// Counts the non-finite values (NaN, +-inf) of n floats into *bad: one atomic per wave.
__global__ __launch_bounds__(256) void count_nonfinite_kernel(const float* x, long long n, int32_t* bad) {
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    const bool nf = i < n && !isfinite(x[i]);
    const unsigned long long m = __ballot(nf);
    if (m != 0ull && __lane_id() == (int)(__ffsll((long long)m) - 1)) atomicAdd(bad, (int32_t)__popcll(m));
}

void launch_count_nonfinite(const float* x, long long n, int32_t* bad, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(count_nonfinite_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, x, n, bad);
}

void launch_adam(const AdamArgs& a, hipStream_t s) {
    if (a.n <= 0) return;
    // sized for the largest group (SH degree >= 1 at degree 3: 45 n values), 4 values a thread
    const long long big = (long long)a.n * (a.sh_k > 1 ? 3 * (a.sh_k - 1) : 4);
    long long g = (big + 1023) / 1024;
    if (g > 8192) g = 8192;
    if (g < 1) g = 1;
    hipLaunchKernelGGL(adam_kernel, dim3((unsigned)g, 6), dim3(256), 0, s, a);
}

// One thread per view (<= AGS_MAX_VIEWS); the exponential map is evaluated in double.
__global__ void pose_step_kernel(ags_camera* cams, int n_views, const float* g, float* m, float* v,
                                 int32_t* step, int advance, float lr, float b1, float b2, float eps) {
    const int b = threadIdx.x;
    const int t = *step;
    __syncthreads();
    if (b < n_views) {
        const double bc1 = 1.0 - pow((double)b1, (double)t);
        const double bc2 = 1.0 - pow((double)b2, (double)t);
        double d[6];
        for (int k = 0; k < 6; ++k) {
            const float gk = g[6 * b + k];
            const float mk = b1 * m[6 * b + k] + (1.f - b1) * gk;
            const float vk = b2 * v[6 * b + k] + (1.f - b2) * gk * gk;
            m[6 * b + k] = mk;
            v[6 * b + k] = vk;
            d[k] = -(double)lr * ((double)mk / bc1) / (sqrt((double)vk / bc2) + (double)eps);
        }
        // Exp(delta): rotation by Rodrigues, translation V rho (left Jacobian of SO(3))
        const double px = d[3], py = d[4], pz = d[5];
        const double th2 = px * px + py * py + pz * pz;
        double A, Bc, Cc;
        if (th2 < 1e-8) {
            A = 1.0 - th2 / 6.0 + th2 * th2 / 120.0;
            Bc = 0.5 - th2 / 24.0 + th2 * th2 / 720.0;
            Cc = 1.0 / 6.0 - th2 / 120.0 + th2 * th2 / 5040.0;
        } else {
            const double th = sqrt(th2);
            A = sin(th) / th;
            Bc = (1.0 - cos(th)) / th2;
            Cc = (th - sin(th)) / (th2 * th);
        }
        const double Kx[9] = {0.0, -pz, py, pz, 0.0, -px, -py, px, 0.0};
        double K2[9];
        for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 3; ++c)
                K2[3 * r + c] = Kx[3 * r] * Kx[c] + Kx[3 * r + 1] * Kx[3 + c] + Kx[3 * r + 2] * Kx[6 + c];
        double Rd[9], V[9];
        for (int k = 0; k < 9; ++k) {
            const double I = (k % 4 == 0) ? 1.0 : 0.0;
            Rd[k] = I + A * Kx[k] + Bc * K2[k];
            V[k] = I + Bc * Kx[k] + Cc * K2[k];
        }
        ags_camera c = cams[b];
        double Rn[9], tn[3];
        for (int r = 0; r < 3; ++r) {
            for (int col = 0; col < 3; ++col)
                Rn[3 * r + col] = Rd[3 * r] * c.R[col] + Rd[3 * r + 1] * c.R[3 + col] + Rd[3 * r + 2] * c.R[6 + col];
            tn[r] = Rd[3 * r] * c.t[0] + Rd[3 * r + 1] * c.t[1] + Rd[3 * r + 2] * c.t[2] +
                    V[3 * r] * d[0] + V[3 * r + 1] * d[1] + V[3 * r + 2] * d[2];
        }
        for (int k = 0; k < 9; ++k) c.R[k] = (float)Rn[k];
        for (int k = 0; k < 3; ++k) c.t[k] = (float)tn[k];
        cams[b] = c;
    }
    __syncthreads();
    if (b == 0 && advance) *step = t + 1;
}

void launch_pose_step(ags_camera* cams, int n_views, const float* g, float* m, float* v,
                      int32_t* step, int advance, float lr, float b1, float b2, float eps,
                      hipStream_t s) {
    hipLaunchKernelGGL(pose_step_kernel, dim3(1), dim3(kMaxViews), 0, s, cams, n_views, g, m, v, step,
                       advance, lr, b1, b2, eps);
}

}  // namespace ags
