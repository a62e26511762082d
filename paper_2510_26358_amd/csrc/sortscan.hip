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

// Apply phase after scan_reduce_kernel's per-block totals: each block adds up the totals of
// the blocks before it (instead of a separate one-workgroup scan of them), writes the
// exclusive scan of its items to out (when non-null), and the last block writes the grand
// total to *total (when non-null).
__global__ __launch_bounds__(kScanThreads) void scan_apply_kernel(
    const uint32_t* src, const uint32_t* idx, bool flags, uint32_t* out, long long n_max,
    const uint32_t* n_dev, const uint32_t* block_sums, uint32_t* total) {
    __shared__ uint32_t wave_tot[kScanThreads / 64];
    const long long n = live_count(n_max, n_dev);
    const long long base = (long long)blockIdx.x * kScanTile;
    if (n == 0 && blockIdx.x == 0 && threadIdx.x == 0 && total) *total = 0u;
    if (base >= n) return;  // uniform per block
    uint32_t pre = 0;
    for (long long b = threadIdx.x; b < (long long)blockIdx.x; b += kScanThreads) pre += block_sums[b];
    uint32_t offset;
    block_inclusive_scan(pre, wave_tot, offset);
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
    if (total && base + kScanTile >= n && threadIdx.x == 0) *total = offset + tot;
    if (!out) return;
    uint32_t run = offset + incl - s;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        long long i = base + (long long)threadIdx.x * kScanItems + k;
        if (i < n) out[i] = run;
        run += v[k];
    }
}

// Scan of the tile counts in depth order (value i = counts[order[i]], i < *n_dev), after
// scan_reduce_kernel's per-block totals: out[i] = offset of item i; for every multiple m of
// kEmitSlots inside item i's range [out[i], out[i] + value) with m < capacity,
// block_first[m / kEmitSlots] = i (the item owning the first slot of that emission
// workgroup; every value is >= 1); and the intersection total, written by the last block:
// counters[CNT_K] = K, counters[CNT_OVERFLOW] = K > capacity, counters[CNT_KEFF] =
// min(K, capacity).
__global__ __launch_bounds__(kScanThreads) void emit_apply_kernel(
    const uint32_t* counts, const uint32_t* order, uint32_t* out, long long n_max, const uint32_t* n_dev,
    const uint32_t* block_sums, long long capacity, uint32_t* block_first, uint32_t* counters) {
    __shared__ uint32_t wave_tot[kScanThreads / 64];
    const long long n = live_count(n_max, n_dev);
    const long long base = (long long)blockIdx.x * kScanTile;
    if (n == 0 && blockIdx.x == 0 && threadIdx.x == 0) {
        counters[CNT_K] = 0u;
        counters[CNT_OVERFLOW] = 0u;
        counters[CNT_KEFF] = 0u;
    }
    if (base >= n) return;  // uniform per block
    // the block's offset: the earlier blocks' totals (at most a few hundred), summed here
    // instead of by a separate scan launch
    uint32_t pre = 0;
    for (long long b = threadIdx.x; b < (long long)blockIdx.x; b += kScanThreads) pre += block_sums[b];
    uint32_t offset;
    block_inclusive_scan(pre, wave_tot, offset);
    uint32_t v[kScanItems];
    uint32_t s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        long long i = base + (long long)threadIdx.x * kScanItems + k;
        v[k] = i < n ? (order ? counts[order[i]] : counts[i]) : 0u;
        s += v[k];
    }
    uint32_t tot;
    uint32_t incl = block_inclusive_scan(s, wave_tot, tot);
    uint32_t run = offset + incl - s;
    if (base + kScanTile >= n && threadIdx.x == 0) {  // the last block holds the grand total
        const uint32_t total = offset + tot;
        const bool over = (long long)total > capacity;
        counters[CNT_K] = total;
        counters[CNT_OVERFLOW] = over ? 1u : 0u;
        counters[CNT_KEFF] = over ? (uint32_t)capacity : total;
    }
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        long long i = base + (long long)threadIdx.x * kScanItems + k;
        if (i < n) {
            out[i] = run;  // out may alias counts: this thread has read its items
            const long long e = (long long)run + v[k];
            for (long long m = ((long long)run + kEmitSlots - 1) / kEmitSlots * kEmitSlots; m < e && m < capacity;
                 m += kEmitSlots)
                block_first[m / kEmitSlots] = (uint32_t)i;
        }
        run += v[k];
    }
}

void launch_emit_scan(const uint32_t* counts, const uint32_t* order, uint32_t* out, long long n_max,
                      const uint32_t* n_dev, uint32_t* counters, long long capacity, uint32_t* block_first,
                      ScanTemp tmp, hipStream_t s) {
    long long nb = scan_blocks(n_max);
    if (nb < 1) nb = 1;
    hipLaunchKernelGGL(scan_reduce_kernel, dim3((unsigned)nb), dim3(kScanThreads), 0, s, counts, order, false,
                       n_max, n_dev, tmp.block_sums);
    hipLaunchKernelGGL(emit_apply_kernel, dim3((unsigned)nb), dim3(kScanThreads), 0, s, counts, order, out, n_max,
                       n_dev, tmp.block_sums, capacity, block_first, counters);
}

void launch_scan(const uint32_t* src, const uint32_t* idx, bool as_flags, uint32_t* out,
                 long long n_max, const uint32_t* n_dev, uint32_t* total, ScanTemp tmp,
                 hipStream_t s) {
    long long nb = scan_blocks(n_max);
    if (nb < 1) nb = 1;
    hipLaunchKernelGGL(scan_reduce_kernel, dim3((unsigned)nb), dim3(kScanThreads), 0, s, src, idx,
                       as_flags, n_max, n_dev, tmp.block_sums);
    if (out || total)
        hipLaunchKernelGGL(scan_apply_kernel, dim3((unsigned)nb), dim3(kScanThreads), 0, s, src,
                           idx, as_flags, out, n_max, n_dev, tmp.block_sums, total);
}

// ------------------------------------------------------------------------- radix sort
// Stable LSD radix sort, up to 8 bits per pass, three kernels per pass (count, scan,
// scatter).  Workgroup b owns the items [b chunk, (b + 1) chunk) of the live count, chunk a
// multiple of the 2048-item tile:
//  1. count: per-workgroup digit totals, stored digit-major (entry d * grid + b).
//  2. row scan: one workgroup per digit turns its row into exclusive offsets and stores
//     the row total.
//  3. scatter: a workgroup starts digit d at (sum of the row totals below d) + its row
//     offset, then per tile ranks the items by digit in LDS and regroups the tile by digit
//     there before writing each digit's run to consecutive addresses.  Each wave ranks a
//     contiguous 512-item slice of the tile, 64 items at a time, against running per-wave
//     digit counts (ballots inside the 64; 4 KB of counts, so six workgroups fit a CU);
//     a scan across waves and digits then places the slices.
// A dropping first pass packs the kept items of successive tiles, in order, into an LDS
// buffer and ranks and writes the buffer whenever the next tile's would not fit, so it ranks
// kept items only (a fifth of the items in the depth sort's pass over every pair), several
// tiles' worth at a time.
// Item order inside a digit is preserved, so the passes compose into a stable sort.
constexpr int kSortThreads = 256;
constexpr int kSortWaves = kSortThreads / 64;
constexpr int kSortItems = 8;                            // items per thread per tile
constexpr int kSortTile = kSortThreads * kSortItems;     // 2048
constexpr int kSortMaxGrid = 4 * kSortThreads;           // row scan: 4 entries per thread

// Workgroups per radix pass: about 8k items each, between 16 and 1024.
int sort_grid(long long n_max) {
    long long g = (n_max + 8191) / 8192;
    return (int)(g < 16 ? 16 : (g > kSortMaxGrid ? kSortMaxGrid : g));
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
    const long long chunk = ((n + grid - 1) / grid + kSortTile - 1) / kSortTile * kSortTile;
    start = (long long)blockIdx.x * chunk;
    end = start + chunk < n ? start + chunk : n;
    if (start > n) start = n;
}

// Exclusive scan of one value per thread over a kSortThreads workgroup; total returned.
__device__ __forceinline__ uint32_t sort_block_scan(uint32_t v, uint32_t* wtot, uint32_t& total) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    uint32_t incl = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(incl, o, 64);
        if (lane >= o) incl += y;
    }
    if (lane == 63) wtot[wv] = incl;
    __syncthreads();
    uint32_t before = 0;
    total = 0;
#pragma unroll
    for (int x = 0; x < kSortWaves; ++x) {
        const uint32_t y = wtot[x];
        before += x < wv ? y : 0u;
        total += y;
    }
    __syncthreads();
    return before + incl - v;
}

__global__ __launch_bounds__(kSortThreads) void radix_count_kernel(
    const uint32_t* keys, long long n_max, const uint32_t* n_dev, int shift, int dbits, uint32_t* hist,
    int grid, bool drop, uint32_t drop_key) {
    __shared__ uint32_t h[256];
    const long long n = live_count(n_max, n_dev);
    long long start, end;
    chunk_of_block(n, grid, start, end);
    h[threadIdx.x] = 0;
    __syncthreads();
    const uint32_t mask = (1u << dbits) - 1u;
    for (long long base = start; base < end; base += kSortTile) {
        uint32_t kv[kSortItems];
#pragma unroll
        for (int k = 0; k < kSortItems; ++k) {
            const long long i = base + k * kSortThreads + threadIdx.x;
            kv[k] = i < end ? keys[i] : 0u;
        }
#pragma unroll
        for (int k = 0; k < kSortItems; ++k) {
            const bool act = base + k * kSortThreads + threadIdx.x < end && !(drop && kv[k] == drop_key);
            const uint32_t dig = (kv[k] >> shift) & mask;
            if (act) atomicAdd(&h[dig], 1u);  // LDS atomics (cheaper here than aggregating by ballots)
        }
    }
    __syncthreads();
    hist[(long long)threadIdx.x * grid + blockIdx.x] = h[threadIdx.x];
}

// Workgroup d: exclusive scan of row d (grid <= kSortMaxGrid entries, 4 consecutive ones per
// thread) in place; row total to rowtot[d].
__global__ __launch_bounds__(kSortThreads) void radix_rowscan_kernel(uint32_t* hist, uint32_t* rowtot,
                                                                     int grid) {
    __shared__ uint32_t wtot[kSortWaves];
    uint32_t* row = hist + (long long)blockIdx.x * grid;
    uint32_t v[4], sum = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int i = 4 * (int)threadIdx.x + k;
        v[k] = i < grid ? row[i] : 0u;
        sum += v[k];
    }
    uint32_t total;
    uint32_t ex = sort_block_scan(sum, wtot, total);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int i = 4 * (int)threadIdx.x + k;
        if (i < grid) row[i] = ex;
        ex += v[k];
    }
    if (threadIdx.x == 0) rowtot[blockIdx.x] = total;
}

template <bool DROP>
__global__ __launch_bounds__(kSortThreads) void radix_scatter_kernel(
    const uint32_t* keys_in, const uint32_t* vals_in, uint32_t* keys_out, uint32_t* vals_out,
    long long n_max, const uint32_t* n_dev, int shift, int dbits, const uint32_t* hist,
    const uint32_t* rowtot, int grid, const uint32_t* gather_src, uint32_t* gather_out,
    uint32_t drop_key, uint32_t* n_live) {
    constexpr int WS = kSortTile / kSortWaves;                // items per wave slice (512)
    __shared__ uint32_t run[256];                             // global cursor per digit
    __shared__ uint32_t wcnt[kSortWaves][256];                // slice counts, then slice bases
    __shared__ uint32_t tstart[256];                          // digit start inside the tile
    __shared__ uint32_t ttot[256];                            // digit count of the tile
    __shared__ uint32_t skey[kSortTile], sval[kSortTile];
    __shared__ uint32_t bkey[DROP ? kSortTile : 1], bval[DROP ? kSortTile : 1];  // kept items, in order
    __shared__ uint32_t wtot[kSortWaves];
    __shared__ uint32_t wkept[kSortWaves];
    const int t = threadIdx.x, w = t >> 6, lane = t & 63;
    // the digit offsets, the live count and then the first tile's items are loaded before the
    // prologue's barriers, so their round trips overlap instead of following one another
    const uint32_t my_rowtot = rowtot[t];
    const uint32_t my_hist = hist[(long long)t * grid + blockIdx.x];
    const long long n = live_count(n_max, n_dev);
    long long start, end;
    chunk_of_block(n, grid, start, end);
    uint32_t kv[kSortItems], vv[kSortItems];
    auto load_tile = [&](long long base) {
        const int nt = end - base < kSortTile ? (int)(end - base) : kSortTile;
#pragma unroll
        for (int k = 0; k < kSortItems; ++k) {
            const int l = w * WS + k * 64 + lane;
            kv[k] = l < nt ? keys_in[base + l] : 0u;
            vv[k] = l < nt ? (vals_in ? vals_in[base + l] : (uint32_t)(base + l)) : 0u;  // index if no values
        }
    };
    if (start < end) load_tile(start);
    {
        uint32_t total;
        const uint32_t base = sort_block_scan(my_rowtot, wtot, total);
        run[t] = base + my_hist;
        if (DROP && n_live && blockIdx.x == 0 && t == 0) *n_live = total;  // items kept
    }
    const uint32_t mask = (1u << dbits) - 1u;
    uint32_t* const cw = wcnt[w];
    // Ranks `cnt` items held `per` to a thread (item k * 64 + lane of wave w's slice of 64 per
    // items is (rk[k], rv[k])), regroups them by digit in LDS and writes each digit's run to
    // its global cursor, which then advances.
    auto rank_write = [&](const uint32_t* rk, const uint32_t* rv, int per, int cnt) {
        uint32_t dig[kSortItems], rank[kSortItems];
        bool on[kSortItems];
#pragma unroll
        for (int x = 0; x < kSortWaves; ++x) wcnt[x][t] = 0;
        __syncthreads();
        // item order inside the slice is (k, lane); the wave's running count of a digit is
        // read by every lane holding it, then advanced by the lowest such lane (LDS
        // operations of one wave complete in issue order)
#pragma unroll
        for (int k = 0; k < kSortItems; ++k) {
            on[k] = k < per && w * 64 * per + k * 64 + lane < cnt;
            dig[k] = (rk[k] >> shift) & mask;
            rank[k] = 0u;
            if (k >= per) continue;  // wave-uniform
            const unsigned long long m = match_digit(dig[k], dbits, __ballot(on[k]));
            const uint32_t below = lanes_below(m);
            const uint32_t prev = on[k] ? cw[dig[k]] : 0u;
            __builtin_amdgcn_wave_barrier();
            if (on[k] && below == 0) cw[dig[k]] = prev + (uint32_t)__popcll(m);
            __builtin_amdgcn_wave_barrier();
            rank[k] = prev + below;
        }
        __syncthreads();
        // thread t = digit: slice bases in wave order, then the digit starts
        uint32_t r = 0;
#pragma unroll
        for (int x = 0; x < kSortWaves; ++x) {
            const uint32_t c = wcnt[x][t];
            wcnt[x][t] = r;
            r += c;
        }
        uint32_t total;  // == cnt
        const uint32_t ds = sort_block_scan(r, wtot, total);
        tstart[t] = ds;
        ttot[t] = r;
        __syncthreads();
#pragma unroll
        for (int k = 0; k < kSortItems; ++k) {
            if (on[k]) {
                const uint32_t pos = tstart[dig[k]] + cw[dig[k]] + rank[k];
                skey[pos] = rk[k];
                sval[pos] = rv[k];
            }
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < kSortItems; ++k) {
            const int p = k * kSortThreads + t;
            if (p < (int)total) {
                const uint32_t key = skey[p];
                const uint32_t d = (key >> shift) & mask;
                const uint32_t dst = run[d] + (uint32_t)p - tstart[d];
                const uint32_t val = sval[p];
                keys_out[dst] = key;
                vals_out[dst] = val;
                if (gather_out) gather_out[dst] = gather_src[val];
            }
        }
        __syncthreads();
        run[t] += ttot[t];
    };
    if (!DROP) {
        for (long long base = start; base < end; base += kSortTile) {
            if (base != start) load_tile(base);
            rank_write(kv, vv, kSortItems, end - base < kSortTile ? (int)(end - base) : kSortTile);
        }
        return;
    }
    // Dropping pass: the kept items of successive tiles are packed, in item order (wave slice,
    // k, lane), into the LDS buffer, and the buffer is ranked and written out whenever the
    // next tile's kept items would not fit (and at the end), so the ranking runs over kept
    // items only, and over several tiles at once when most items are dropped.
    int buffered = 0;  // workgroup-uniform
    uint32_t bk[kSortItems], bv[kSortItems];
    auto flush = [&]() {
        const int per = (buffered + kSortThreads - 1) / kSortThreads;
#pragma unroll
        for (int k = 0; k < kSortItems; ++k) {
            const int j = w * 64 * per + k * 64 + lane;
            const bool in = k < per && j < buffered;
            bk[k] = in ? bkey[j] : 0u;
            bv[k] = in ? bval[j] : 0u;
        }
        rank_write(bk, bv, per, buffered);
        buffered = 0;
    };
    for (long long base = start; base < end; base += kSortTile) {
        const int nt = end - base < kSortTile ? (int)(end - base) : kSortTile;
        if (base != start) load_tile(base);
        uint32_t wk = 0, pw[kSortItems];
        bool keep[kSortItems];
#pragma unroll
        for (int k = 0; k < kSortItems; ++k) {
            keep[k] = w * WS + k * 64 + lane < nt && kv[k] != drop_key;
            const unsigned long long b = __ballot(keep[k]);
            pw[k] = wk + lanes_below(b);
            wk += (uint32_t)__popcll(b);
        }
        if (lane == 0) wkept[w] = wk;
        __syncthreads();
        uint32_t woff = 0, nk = 0;
#pragma unroll
        for (int x = 0; x < kSortWaves; ++x) {
            const uint32_t c = wkept[x];
            woff += x < w ? c : 0u;
            nk += c;
        }
        if (buffered + (int)nk > kSortTile) flush();  // its barriers also order the wkept reads
#pragma unroll
        for (int k = 0; k < kSortItems; ++k)
            if (keep[k]) {
                bkey[buffered + woff + pw[k]] = kv[k];
                bval[buffered + woff + pw[k]] = vv[k];
            }
        buffered += (int)nk;
        __syncthreads();
    }
    if (buffered > 0) flush();
}

int launch_radix_sort(uint32_t* keys[2], uint32_t* vals[2], long long n_max, const uint32_t* n_dev,
                      int bits, int grid, SortTemp tmp, hipStream_t s, const uint32_t* gather_src,
                      uint32_t* gather_out, uint32_t* n_live, uint32_t drop_key, const uint32_t* first_keys) {
    const int passes = sort_passes(bits);
    if (passes == 0) return 0;
    const int dbits = (bits + passes - 1) / passes;
    // pass p reads buffer `in` and writes buffer `out`; with first_keys the first pass reads
    // the external keys (values = indices) and writes buffer 0
    int in = 0;
    for (int p = 0; p < passes; ++p) {
        const int shift = p * dbits;
        const int db = (shift + dbits > bits) ? bits - shift : dbits;
        const bool drop = n_live && p == 0;
        // after a dropping first pass the later ones sort only the items kept
        const uint32_t* nd = (n_live && p > 0) ? n_live : n_dev;
        const bool ext = first_keys && p == 0;
        const uint32_t* kin = ext ? first_keys : keys[in];
        const uint32_t* vin = ext ? nullptr : vals[in];
        const int out = ext ? 0 : 1 - in;
        hipLaunchKernelGGL(radix_count_kernel, dim3(grid), dim3(kSortThreads), 0, s, kin, n_max, nd, shift, db,
                           tmp.hist, grid, drop, drop_key);
        hipLaunchKernelGGL(radix_rowscan_kernel, dim3(256), dim3(kSortThreads), 0, s, tmp.hist, tmp.rowtot, grid);
        if (drop)
            hipLaunchKernelGGL(radix_scatter_kernel<true>, dim3(grid), dim3(kSortThreads), 0, s, kin, vin,
                               keys[out], vals[out], n_max, nd, shift, db, tmp.hist, tmp.rowtot, grid,
                               p == passes - 1 ? gather_src : nullptr, p == passes - 1 ? gather_out : nullptr,
                               drop_key, n_live);
        else
            hipLaunchKernelGGL(radix_scatter_kernel<false>, dim3(grid), dim3(kSortThreads), 0, s, kin, vin,
                               keys[out], vals[out], n_max, nd, shift, db, tmp.hist, tmp.rowtot, grid,
                               p == passes - 1 ? gather_src : nullptr, p == passes - 1 ? gather_out : nullptr,
                               drop_key, n_live);
        in = out;
    }
    return in;
}

long long sort_hist_entries(int grid) { return 256LL * grid; }
long long sort_rowtot_entries() { return 256; }

}  // namespace ags
