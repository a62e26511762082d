// Device-wide primitives: fills, exclusive scan and a stable LSD radix sort of
// (uint32 key, uint32 value) pairs.  Element counts may live in device memory so the
// whole forward can be enqueued (and graph-captured) without a host round trip: grids
// are sized for the static maximum and blocks past the live count do nothing.
#include "common.h"

namespace ags {

// ------------------------------------------------------------------------- fills
__global__ void fill_u32_kernel(uint32_t* p, uint32_t v, long long n) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    long long stride = (long long)gridDim.x * blockDim.x;
    for (; i < n; i += stride) p[i] = v;
}
__global__ void fill_f32_kernel(float* p, float v, long long n) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    long long stride = (long long)gridDim.x * blockDim.x;
    for (; i < n; i += stride) p[i] = v;
}
static int fill_grid(long long n) {
    long long g = (n + 255) / 256;
    return (int)(g < 1 ? 1 : (g > 8192 ? 8192 : g));
}
void launch_fill_u32(uint32_t* p, uint32_t v, long long n, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(fill_u32_kernel, dim3(fill_grid(n)), dim3(256), 0, s, p, v, n);
}
void launch_fill_f32(float* p, float v, long long n, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(fill_f32_kernel, dim3(fill_grid(n)), dim3(256), 0, s, p, v, n);
}

// ------------------------------------------------------------------------- scan
constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr int kScanTile = kScanThreads * kScanItems;

long long scan_blocks(long long n_max) { return (n_max + kScanTile - 1) / kScanTile; }

__device__ __forceinline__ long long live_count(long long n_max, const uint32_t* n_dev) {
    if (!n_dev) return n_max;
    long long n = (long long)(*n_dev);
    return n < n_max ? n : n_max;
}

__device__ __forceinline__ uint32_t scan_value(const uint32_t* src, const uint32_t* idx,
                                               bool flags, long long i) {
    uint32_t v = idx ? src[idx[i]] : src[i];
    return flags ? (v != 0u ? 1u : 0u) : v;
}

// Inclusive scan of one value per thread across a 256-thread block; returns the block
// total through `total`.
__device__ __forceinline__ uint32_t block_inclusive_scan(uint32_t v, uint32_t* wave_tot,
                                                         uint32_t& total) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        uint32_t t = __shfl_up(v, o, 64);
        if (lane >= o) v += t;
    }
    if (lane == 63) wave_tot[wave] = v;
    __syncthreads();
    uint32_t add = 0;
    total = 0;
#pragma unroll
    for (int w = 0; w < kScanThreads / 64; ++w) {
        uint32_t t = wave_tot[w];
        if (w < wave) add += t;
        total += t;
    }
    __syncthreads();
    return v + add;
}

__global__ __launch_bounds__(kScanThreads) void scan_reduce_kernel(
    const uint32_t* src, const uint32_t* idx, bool flags, long long n_max, const uint32_t* n_dev,
    uint32_t* block_sums) {
    __shared__ uint32_t wave_tot[kScanThreads / 64];
    const long long n = live_count(n_max, n_dev);
    const long long base = (long long)blockIdx.x * kScanTile;
    uint32_t s = 0;
    if (base < n) {
#pragma unroll
        for (int k = 0; k < kScanItems; ++k) {
            long long i = base + (long long)k * kScanThreads + threadIdx.x;
            if (i < n) s += scan_value(src, idx, flags, i);
        }
    }
    uint32_t total;
    block_inclusive_scan(s, wave_tot, total);
    if (threadIdx.x == 0) block_sums[blockIdx.x] = total;
}

// Single block: exclusive scan of the block sums in place; grand total to *total.
__global__ __launch_bounds__(kScanThreads) void scan_blocksums_kernel(uint32_t* block_sums,
                                                                      long long nb, uint32_t* total) {
    __shared__ uint32_t wave_tot[kScanThreads / 64];
    uint32_t carry = 0;
    for (long long base = 0; base < nb; base += kScanTile) {
        uint32_t v[kScanItems];
        uint32_t s = 0;
#pragma unroll
        for (int k = 0; k < kScanItems; ++k) {
            long long i = base + (long long)threadIdx.x * kScanItems + k;
            v[k] = i < nb ? block_sums[i] : 0u;
            s += v[k];
        }
        uint32_t tot;
        uint32_t incl = block_inclusive_scan(s, wave_tot, tot);
        uint32_t run = carry + incl - s;
#pragma unroll
        for (int k = 0; k < kScanItems; ++k) {
            long long i = base + (long long)threadIdx.x * kScanItems + k;
            if (i < nb) block_sums[i] = run;
            run += v[k];
        }
        carry += tot;
    }
    if (threadIdx.x == 0 && total) *total = carry;
}

__global__ __launch_bounds__(kScanThreads) void scan_apply_kernel(
    const uint32_t* src, const uint32_t* idx, bool flags, uint32_t* out, long long n_max,
    const uint32_t* n_dev, const uint32_t* block_sums) {
    __shared__ uint32_t wave_tot[kScanThreads / 64];
    const long long n = live_count(n_max, n_dev);
    const long long base = (long long)blockIdx.x * kScanTile;
    if (base >= n) return;  // uniform per block
    uint32_t v[kScanItems];
    uint32_t s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        long long i = base + (long long)threadIdx.x * kScanItems + k;
        v[k] = i < n ? scan_value(src, idx, flags, i) : 0u;
        s += v[k];
    }
    uint32_t tot;
    uint32_t incl = block_inclusive_scan(s, wave_tot, tot);
    uint32_t run = block_sums[blockIdx.x] + incl - s;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        long long i = base + (long long)threadIdx.x * kScanItems + k;
        if (i < n) out[i] = run;
        run += v[k];
    }
}

// Apply phase that compacts instead of writing prefixes: element i with src[i] != 0 goes to
// position prefix(i) of (keys, vals) as (payload[i], i).  Order-preserving.
__global__ __launch_bounds__(kScanThreads) void scan_compact_kernel(
    const uint32_t* src, const uint32_t* payload, long long n, const uint32_t* block_sums, uint32_t* keys,
    uint32_t* vals) {
    __shared__ uint32_t wave_tot[kScanThreads / 64];
    const long long base = (long long)blockIdx.x * kScanTile;
    if (base >= n) return;
    uint32_t v[kScanItems];
    uint32_t s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        long long i = base + (long long)threadIdx.x * kScanItems + k;
        v[k] = (i < n && src[i] != 0u) ? 1u : 0u;
        s += v[k];
    }
    uint32_t tot;
    uint32_t incl = block_inclusive_scan(s, wave_tot, tot);
    uint32_t run = block_sums[blockIdx.x] + incl - s;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        long long i = base + (long long)threadIdx.x * kScanItems + k;
        if (v[k]) {
            keys[run] = payload[i];
            vals[run] = (uint32_t)i;
        }
        run += v[k];
    }
}

void launch_scan_compact(const uint32_t* src, const uint32_t* payload, long long n, uint32_t* total,
                         uint32_t* keys, uint32_t* vals, ScanTemp tmp, hipStream_t s) {
    long long nb = scan_blocks(n);
    if (nb < 1) nb = 1;
    hipLaunchKernelGGL(scan_reduce_kernel, dim3((unsigned)nb), dim3(kScanThreads), 0, s, src, nullptr, true, n,
                       nullptr, tmp.block_sums);
    hipLaunchKernelGGL(scan_blocksums_kernel, dim3(1), dim3(kScanThreads), 0, s, tmp.block_sums, nb, total);
    hipLaunchKernelGGL(scan_compact_kernel, dim3((unsigned)nb), dim3(kScanThreads), 0, s, src, payload, n,
                       tmp.block_sums, keys, vals);
}

void launch_scan(const uint32_t* src, const uint32_t* idx, bool as_flags, uint32_t* out,
                 long long n_max, const uint32_t* n_dev, uint32_t* total, ScanTemp tmp,
                 hipStream_t s) {
    long long nb = scan_blocks(n_max);
    if (nb < 1) nb = 1;
    hipLaunchKernelGGL(scan_reduce_kernel, dim3((unsigned)nb), dim3(kScanThreads), 0, s, src, idx,
                       as_flags, n_max, n_dev, tmp.block_sums);
    hipLaunchKernelGGL(scan_blocksums_kernel, dim3(1), dim3(kScanThreads), 0, s, tmp.block_sums,
                       nb, total);
    if (out)
        hipLaunchKernelGGL(scan_apply_kernel, dim3((unsigned)nb), dim3(kScanThreads), 0, s, src,
                           idx, as_flags, out, n_max, n_dev, tmp.block_sums);
}

// ------------------------------------------------------------------------- radix sort
constexpr int kSortThreads = 256;
constexpr int kSortWaves = kSortThreads / 64;
constexpr int kSortMaxGrid = 1024;

// Workgroups per radix pass: about 8k items each, between 64 and 1024.
int sort_grid(long long n_max) {
    long long g = (n_max + 8191) / 8192;
    return (int)(g < 64 ? 64 : (g > kSortMaxGrid ? kSortMaxGrid : g));
}
int sort_passes(int bits) { return bits <= 0 ? 0 : (bits + 7) / 8; }

// Lanes of the calling wave holding the same digit as this lane (among `active` lanes),
// found with one ballot per digit bit.
__device__ __forceinline__ unsigned long long match_digit(uint32_t dig, int dbits,
                                                          unsigned long long active) {
    unsigned long long m = active;
    for (int b = 0; b < dbits; ++b) {
        unsigned long long bal = __ballot((dig >> b) & 1u);
        m &= ((dig >> b) & 1u) ? bal : ~bal;
    }
    return m;
}

__device__ __forceinline__ uint32_t lanes_below(unsigned long long m) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

__device__ __forceinline__ void chunk_of_block(long long n, int grid, long long& start, long long& end) {
    long long chunk = (n + grid - 1) / grid;
    start = (long long)blockIdx.x * chunk;
    end = start + chunk;
    if (end > n) end = n;
}

__global__ __launch_bounds__(kSortThreads) void radix_hist_kernel(
    const uint32_t* keys, long long n_max, const uint32_t* n_dev, int shift, int dbits,
    uint32_t* hist, int grid) {
    __shared__ uint32_t h[256];
    const long long n = live_count(n_max, n_dev);
    long long start, end;
    chunk_of_block(n, grid, start, end);
    h[threadIdx.x] = 0;
    __syncthreads();
    const uint32_t mask = (1u << dbits) - 1u;
    for (long long base = start; base < end; base += kSortThreads) {
        long long i = base + threadIdx.x;
        bool act = i < end;
        uint32_t dig = act ? (keys[i] >> shift) & mask : 0u;
        unsigned long long active = __ballot(act);
        unsigned long long m = match_digit(dig, dbits, active);
        if (act && lanes_below(m) == 0) atomicAdd(&h[dig], (uint32_t)__popcll(m));
    }
    __syncthreads();
    hist[(long long)threadIdx.x * grid + blockIdx.x] = h[threadIdx.x];
}

__global__ __launch_bounds__(kSortThreads) void radix_scatter_kernel(
    const uint32_t* keys_in, const uint32_t* vals_in, uint32_t* keys_out, uint32_t* vals_out,
    long long n_max, const uint32_t* n_dev, int shift, int dbits, const uint32_t* hist_scanned,
    int grid) {
    __shared__ uint32_t run[256];
    __shared__ uint32_t wcnt[kSortWaves][256];
    const long long n = live_count(n_max, n_dev);
    long long start, end;
    chunk_of_block(n, grid, start, end);
    const int wave = threadIdx.x >> 6;
    run[threadIdx.x] = hist_scanned[(long long)threadIdx.x * grid + blockIdx.x];
    const uint32_t mask = (1u << dbits) - 1u;
    for (long long base = start; base < end; base += kSortThreads) {
#pragma unroll
        for (int w = 0; w < kSortWaves; ++w) wcnt[w][threadIdx.x] = 0;
        __syncthreads();
        long long i = base + threadIdx.x;
        bool act = i < end;
        uint32_t key = act ? keys_in[i] : 0u;
        uint32_t val = act ? vals_in[i] : 0u;
        uint32_t dig = (key >> shift) & mask;
        unsigned long long active = __ballot(act);
        unsigned long long m = match_digit(dig, dbits, active);
        uint32_t below = lanes_below(m);
        if (act && below == 0) wcnt[wave][dig] = (uint32_t)__popcll(m);
        __syncthreads();
        if (act) {
            uint32_t r = run[dig] + below;
            for (int w = 0; w < wave; ++w) r += wcnt[w][dig];
            keys_out[r] = key;
            vals_out[r] = val;
        }
        __syncthreads();
        uint32_t add = 0;
#pragma unroll
        for (int w = 0; w < kSortWaves; ++w) add += wcnt[w][threadIdx.x];
        run[threadIdx.x] += add;
        __syncthreads();
    }
}

int launch_radix_sort(uint32_t* keys[2], uint32_t* vals[2], long long n_max, const uint32_t* n_dev,
                      int bits, SortTemp tmp, hipStream_t s) {
    const int passes = sort_passes(bits);
    if (passes == 0) return 0;
    const int dbits = (bits + passes - 1) / passes;
    const int grid = tmp.grid;
    int cur = 0;
    ScanTemp st{tmp.hist_sums};
    for (int p = 0; p < passes; ++p) {
        const int shift = p * dbits;
        const int db = (shift + dbits > bits) ? bits - shift : dbits;
        hipLaunchKernelGGL(radix_hist_kernel, dim3(grid), dim3(kSortThreads), 0, s, keys[cur], n_max,
                           n_dev, shift, db, tmp.hist, grid);
        launch_scan(tmp.hist, nullptr, false, tmp.hist, 256LL * grid, nullptr, nullptr, st, s);
        hipLaunchKernelGGL(radix_scatter_kernel, dim3(grid), dim3(kSortThreads), 0, s, keys[cur],
                           vals[cur], keys[1 - cur], vals[1 - cur], n_max, n_dev, shift, db, tmp.hist,
                           grid);
        cur = 1 - cur;
    }
    return cur;
}

}  // namespace ags
