// Gaussian-splat lifecycle operations (Sec. III-B, "Gaussian Splats Lifecycle Operations"):
// pruning, gradient-driven densification (split / duplicate) and opacity reset, as an
// order-preserving stream compaction over the structure-of-arrays parameters and their
// Adam moments.
//
// 1. classify: one thread per Gaussian decides keep / prune / duplicate / split (float32,
//    the rules of ags_lifecycle in agsplat.h) and its number of outputs (0, 1 or 2);
// 2. exclusive scan of the output counts -> first output slot, total -> *n_out;
// 3. scatter: one thread per surviving Gaussian writes its outputs into every row of the
//    output arrays; split children get mu + R(q) diag(s) eps and log-scales - ln(split_scale),
//    copies and children zero Adam moments, survivors keep theirs.
#include "common.h"

namespace ags {

enum { LC_KEEP = 0, LC_PRUNE = 1, LC_CLONE = 2, LC_SPLIT = 3 };

__global__ void lifecycle_classify_kernel(LifecycleArgs a) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.n) return;
    const int n = a.n;
    const float* ls = a.in[0][1];
    const float o = 1.f / (1.f + expf(-a.in[0][3][i]));
    const float s = expf(fmaxf(fmaxf(ls[i], ls[n + i]), ls[2 * n + i]));
    int act = LC_KEEP;
    if (a.do_prune && (o < a.tau_opa || s > a.s_max || s < a.s_min)) act = LC_PRUNE;
    if (act == LC_KEEP && a.do_densify) {
        const float c = a.stat_count[i];
        const float g = a.stat_grad[i] / fmaxf(c, 1.f);
        if (c > 0.f && g > a.grad_threshold) {
            if (s > a.kappa) act = LC_SPLIT;
            else if (s <= a.two_s_init) act = LC_CLONE;
        }
    }
    a.counts[i] = act == LC_PRUNE ? 0u : (act == LC_KEEP ? 1u : 2u);
    if (a.actions) a.actions[i] = (uint8_t)act;
}

__global__ void lifecycle_scatter_kernel(LifecycleArgs a) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.n) return;
    const uint32_t cnt = a.counts[i];
    if (cnt == 0) return;
    const int n = a.n;
    const long long cap = a.cap;
    const long long j0 = a.offsets[i];
    const float* ls = a.in[0][1];
    const float o = 1.f / (1.f + expf(-a.in[0][3][i]));
    const float smax = expf(fmaxf(fmaxf(ls[i], ls[n + i]), ls[2 * n + i]));
    const bool reset = a.do_reset && o >= a.tau_opa && o < a.tau_reset && smax >= a.s_min && smax <= a.s_max;
    const float logit = reset ? a.reset_logit : a.in[0][3][i];
    bool split = false;
    if (cnt == 2) {  // duplicate or split: the size test tells them apart as in classify
        split = smax > a.kappa;
    }
    // rows: [0] means (3), [1] log_scales (3), [2] quats (4), [3] logits (1), [4] sh (k3)
    const int rows[5] = {3, 3, 4, 1, a.k3};
    for (uint32_t c = 0; c < cnt; ++c) {
        const long long j = j0 + c;
        const bool fresh = c == 1 || split;  // copies and children start with zero moments
        for (int f = 0; f < 5; ++f) {
            for (int r = 0; r < rows[f]; ++r) {
                float val = a.in[0][f][(long long)r * n + i];
                if (f == 3) val = logit;
                a.out[0][f][(long long)r * cap + j] = val;
                a.out[1][f][(long long)r * cap + j] = fresh ? 0.f : a.in[1][f][(long long)r * n + i];
                a.out[2][f][(long long)r * cap + j] = fresh ? 0.f : a.in[2][f][(long long)r * n + i];
            }
        }
        if (split) {
            const float* q = a.in[0][2];
            float qw = q[i], qx = q[n + i], qy = q[2 * n + i], qz = q[3 * n + i];
            const float qi = rsqrtf(qw * qw + qx * qx + qy * qy + qz * qz);
            float R[9];
            quat_to_rot(qw * qi, qx * qi, qy * qi, qz * qi, R);
            const float sc[3] = {expf(ls[i]), expf(ls[n + i]), expf(ls[2 * n + i])};
            const float* e = a.noise + ((long long)i * 2 + c) * 3;
            const float d[3] = {sc[0] * e[0], sc[1] * e[1], sc[2] * e[2]};
            for (int r = 0; r < 3; ++r) {
                a.out[0][0][(long long)r * cap + j] =
                    a.in[0][0][(long long)r * n + i] + R[3 * r] * d[0] + R[3 * r + 1] * d[1] + R[3 * r + 2] * d[2];
                a.out[0][1][(long long)r * cap + j] = ls[(long long)r * n + i] - a.log_split;
            }
        }
    }
}

void launch_lifecycle(const LifecycleArgs& a, hipStream_t s) {
    if (a.n <= 0) {
        launch_fill_u32(reinterpret_cast<uint32_t*>(a.n_out), 0u, 1, s);
        return;
    }
    const unsigned grid = (unsigned)((a.n + 255) / 256);
    hipLaunchKernelGGL(lifecycle_classify_kernel, dim3(grid), dim3(256), 0, s, a);
    launch_scan(a.counts, nullptr, false, a.offsets, a.n, nullptr, reinterpret_cast<uint32_t*>(a.n_out),
                a.scan_tmp, s);
    hipLaunchKernelGGL(lifecycle_scatter_kernel, dim3(grid), dim3(256), 0, s, a);
}

}  // namespace ags
