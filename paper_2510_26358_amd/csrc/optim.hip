// Joint refinement updates: Adam on the Gaussian parameters and Adam on each camera's
// se(3) increment followed by the left retraction W <- Exp(delta) W.  The paper refines
// splats and poses jointly by gradient steps on the multimodal loss (Sec. III-C); Adam and
// the tangent-space pose update are the refinement workload's choice.  The step number is
// read from device memory so a captured optimisation step can be replayed unchanged.
#include "common.h"

namespace ags {

__global__ __launch_bounds__(256) void adam_kernel(AdamArgs a) {
    const long long n = a.n;
    const long long sizes[5] = {3 * n, 3 * n, 4 * n, n, (long long)a.sh_k * 3 * n};
    const long long total = sizes[0] + sizes[1] + sizes[2] + sizes[3] + sizes[4];
    const float t = (float)(*a.step);
    const float bc1 = 1.f - powf(a.beta1, t);
    const float bc2 = 1.f - powf(a.beta2, t);
    long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (; e < total; e += stride) {
        long long j = e;
        int seg = 0;
        while (seg < 4 && j >= sizes[seg]) {
            j -= sizes[seg];
            ++seg;
        }
        const float lr = seg < 4 ? a.lr[seg] : (j < 3 * n ? a.lr[4] : a.lr[5]);
        const float g = a.g[seg][j];
        const float m = a.beta1 * a.m[seg][j] + (1.f - a.beta1) * g;
        const float v = a.beta2 * a.v[seg][j] + (1.f - a.beta2) * g * g;
        a.m[seg][j] = m;
        a.v[seg][j] = v;
        a.p[seg][j] -= lr * (m / bc1) / (sqrtf(v / bc2) + a.eps);
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
    long long total = (long long)a.n * (11 + 3 * a.sh_k);
    long long g = (total + 255) / 256;
    if (g > 16384) g = 16384;
    hipLaunchKernelGGL(adam_kernel, dim3((unsigned)g), dim3(256), 0, s, a);
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
