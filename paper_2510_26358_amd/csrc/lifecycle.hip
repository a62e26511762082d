// Gaussian-splat lifecycle operations (Sec. III-B, "Gaussian Splats Lifecycle Operations"):
// pruning, gradient-driven densification (split / duplicate) and opacity reset, as an
// order-preserving stream compaction over the structure-of-arrays parameters and their
// Adam moments.
//
// 1. classify: one thread per Gaussian decides keep / prune / duplicate / split (float32,
//    the rules of ags_lifecycle in agsplat.h) and its number of outputs (0, 1 or 2);
// 2. exclusive scan of the output counts -> first output slot, total -> *n_out;
// 3. scatter: a thread per surviving Gaussian and group of rows (of the parameters or one of
//    the moment arrays) loads the rows, then writes the Gaussian's outputs; split children get
//    mu + R(q) diag(s) eps and log-scales - ln(split_scale), copies and children zero Adam
//    moments, survivors keep theirs.
#include <mutex>

#include "common.h"

namespace ags {

namespace {

// Scratch of ags_lifecycle_step_noalloc: a static device array, one copy on every GPU the
// library runs on, alive until the process ends.  In host code `scratch` names a host-side
// stand-in, not device memory: its device address comes from hipGetSymbolAddress, looked up
// once per device (lifecycle_static_scratch) and passed to the kernels like a workspace.
constexpr size_t kStaticScratchBytes = (size_t)AGS_LIFECYCLE_NOALLOC_BYTES;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices];

}  // namespace

int lifecycle_static_scratch(int device, void** ptr, size_t* bytes) {
    if (device < 0 || device >= kMaxDevices || !ptr || !bytes) return AGS_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        int cur = -1;
        if (hipGetDevice(&cur) != hipSuccess) return AGS_ERR_HIP;
        if (cur != device && hipSetDevice(device) != hipSuccess) return AGS_ERR_HIP;
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (cur != device) (void)hipSetDevice(cur);
        if (e != hipSuccess || !p) return AGS_ERR_HIP;
        g_scratch_ptr[device] = p;
    }
    *ptr = g_scratch_ptr[device];
    *bytes = kStaticScratchBytes;
    return AGS_OK;
}

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

constexpr int kLcRows = 16;  // SH rows one thread moves per launch row

// Split flag of a Gaussian with two outputs (duplicate and split differ only by size).
__device__ __forceinline__ bool lc_is_split(const LifecycleArgs& a, int i) {
    const float* ls = a.in[0][1];
    const int n = a.n;
    return expf(fmaxf(fmaxf(ls[i], ls[n + i]), ls[2 * n + i])) > a.kappa;
}

// Copies `rows` rows (row stride n in, cap out) of one field for Gaussian i: all loads are
// issued before the first store (the row index is clamped, not branched on).
template <int R>
__device__ __forceinline__ void lc_copy(const float* __restrict__ src, float* __restrict__ dst, int rows, int n,
                                        long long cap, int i, long long j0, uint32_t cnt, bool zero0, bool zero1) {
    float v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) v[r] = src[(long long)(r < rows ? r : rows - 1) * n + i];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        if (r < rows) {
            dst[(long long)r * cap + j0] = zero0 ? 0.f : v[r];
            if (cnt == 2) dst[(long long)r * cap + j0 + 1] = zero1 ? 0.f : v[r];
        }
    }
}

// grid (ceil(n / 256), 3 * lc_chunks): blockIdx.y = array (params, m, v) x chunk, chunk 0 =
// means / log-scales / quaternion / logit, chunks 1.. = SH rows in groups of kLcRows.
__global__ __launch_bounds__(256) void lifecycle_scatter_kernel(LifecycleArgs a) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.n) return;
    const uint32_t cnt = a.counts[i];
    if (cnt == 0) return;
    const int n = a.n;
    const long long cap = a.cap;
    const long long j0 = a.offsets[i];
    const int t = blockIdx.y / a.chunks, c = blockIdx.y % a.chunks;
    if (t == 0 && c == 0) {
        // parameters: split children and the opacity reset
        const float* ls = a.in[0][1];
        const float* mu = a.in[0][0];
        const float* q = a.in[0][2];
        const float l0 = ls[i], l1 = ls[n + i], l2 = ls[2 * n + i];
        const float m0 = mu[i], m1 = mu[n + i], m2 = mu[2 * n + i];
        const float qw = q[i], qx = q[n + i], qy = q[2 * n + i], qz = q[3 * n + i];
        const float lg = a.in[0][3][i];
        const float o = 1.f / (1.f + expf(-lg));
        const float smax = expf(fmaxf(fmaxf(l0, l1), l2));
        const bool reset = a.do_reset && o >= a.tau_opa && o < a.tau_reset && smax > a.s_min && smax < a.s_max;
        const float logit = reset ? a.reset_logit : lg;
        const bool split = cnt == 2 && smax > a.kappa;
        float* const* out = a.out[0];
        float mo[2][3] = {{m0, m1, m2}, {m0, m1, m2}};
        float lo[3] = {l0, l1, l2};
        if (split) {
            const float qi = rsqrtf(qw * qw + qx * qx + qy * qy + qz * qz);
            float R[9];
            quat_to_rot(qw * qi, qx * qi, qy * qi, qz * qi, R);
            const float sc[3] = {expf(l0), expf(l1), expf(l2)};
            const float* e = a.noise + (long long)i * 6;
            for (int k = 0; k < 2; ++k) {
                const float d[3] = {sc[0] * e[3 * k], sc[1] * e[3 * k + 1], sc[2] * e[3 * k + 2]};
                for (int r = 0; r < 3; ++r)
                    mo[k][r] += R[3 * r] * d[0] + R[3 * r + 1] * d[1] + R[3 * r + 2] * d[2];
            }
            for (int r = 0; r < 3; ++r) lo[r] -= a.log_split;
        }
        const float qv[4] = {qw, qx, qy, qz};
        for (uint32_t k = 0; k < cnt; ++k) {
            const long long j = j0 + k;
            for (int r = 0; r < 3; ++r) {
                out[0][r * cap + j] = mo[k][r];
                out[1][r * cap + j] = lo[r];
            }
            for (int r = 0; r < 4; ++r) out[2][r * cap + j] = qv[r];
            out[3][j] = logit;
        }
        return;
    }
    // copies and children start with zero Adam moments; survivors keep theirs
    bool zero0 = false, zero1 = false;
    if (t > 0 && cnt == 2) {
        zero1 = true;
        zero0 = lc_is_split(a, i);
    }
    if (c == 0) {
        const int rows[4] = {3, 3, 4, 1};
#pragma unroll
        for (int f = 0; f < 4; ++f)
            lc_copy<4>(a.in[t][f], a.out[t][f], rows[f], n, cap, i, j0, cnt, zero0, zero1);
        return;
    }
    const int r0 = (c - 1) * kLcRows;
    const int rows = a.k3 - r0 < kLcRows ? a.k3 - r0 : kLcRows;
    lc_copy<kLcRows>(a.in[t][4] + (long long)r0 * n, a.out[t][4] + (long long)r0 * cap, rows, n, cap, i, j0, cnt,
                     zero0, zero1);
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
    LifecycleArgs b = a;
    b.chunks = 1 + (a.k3 + kLcRows - 1) / kLcRows;
    hipLaunchKernelGGL(lifecycle_scatter_kernel, dim3(grid, 3 * b.chunks), dim3(256), 0, s, b);
}

}  // namespace ags
