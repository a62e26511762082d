// Tile binning: per-tile Gaussian lists in depth order, for all views at once.
//
// Order definition: every (view b, Gaussian i, tile) intersection carries the key
// (global tile, float32 depth bits) and the lists are the stable ascending order of those
// keys over emission order (b, i, ty, tx) -- ties resolve by ascending pair id.
//
// Instead of radix-sorting 64-bit keys over all K intersections, the visible pairs are
// depth-sorted once (V << K items, 32-bit keys) and their intersections are emitted in
// that order; a stable sort on the tile id alone then yields exactly the same order
// (LSD radix passes are stable).  Bytes moved: 4 passes x V + ceil(tile_bits / 8) passes
// x K instead of 6 passes x K with 12-byte records.
#include "common.h"

namespace ags {

// Emission.  Output slot k belongs to the last pair j (depth order) with emit_off[j] <= k and
// is slot k - emit_off[j] of that pair's tile rectangle (row-major).  A workgroup fills
// kEmitSlots consecutive slots; since every visible pair owns >= 1 slot, they belong to at
// most kEmitSlots consecutive pairs starting at block_first[workgroup].  Their offsets, and
// for each pair the rectangle's first tile, its width, the view and the ellipse (centre,
// conic, level), are staged in LDS (one thread per pair); each pair marks its first slot
// and a prefix maximum over the slots gives every slot its pair.  A slot whose tile the
// alpha >= alpha_min ellipse does not reach (tile_reached) gets the key n_tiles, which the
// tile sort's first pass drops.  Balanced however unequal the footprints are, and the
// writes are coalesced.
constexpr int kEmitThreads = 256;

__global__ __launch_bounds__(kEmitThreads) void emit_kernel(ViewTable vt, const float* records,
                                                            const uint32_t* depth_vals, const uint32_t* emit_off,
                                                            const uint32_t* block_first, const uint32_t* counters,
                                                            long long capacity, uint32_t* tile_keys,
                                                            uint32_t* tile_vals, uint32_t* ranges) {
    constexpr int S = kEmitSlots, PT = S / kEmitThreads;
    __shared__ uint32_t s_off[S];
    __shared__ uint32_t s_own[S];                     // slot -> local pair index
    __shared__ uint32_t s_q[S], s_first[S];           // pair, global id of the rectangle's first tile
    __shared__ uint32_t s_wp[S], s_org[S], s_wh[S];   // width | pitch << 16, tx0 | ty0 << 16, W | H << 16
    __shared__ float4 s_ell[S];                       // u, v, a, b
    __shared__ float2 s_ell2[S];                      // c, level
    __shared__ uint32_t s_wmax[kEmitThreads / 64];
    const long long k0 = (long long)blockIdx.x * S;
    const uint32_t n_tiles = (uint32_t)vt.tile_base[vt.n_views];
    // every tile's range starts empty; ranges_kernel later sets the non-empty ones
    for (long long e = (long long)blockIdx.x * kEmitThreads + threadIdx.x; e < 2LL * n_tiles;
         e += (long long)gridDim.x * kEmitThreads)
        ranges[e] = 0u;
    long long keff = counters[CNT_KEFF];
    if (keff > capacity) keff = capacity;
    const long long nv = counters[CNT_V];
    if (k0 >= keff || nv == 0) return;  // uniform per workgroup
    const long long j0 = block_first[blockIdx.x];
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    // the workgroup's pairs: from the owner of its first slot to the owner of the next
    // workgroup's first slot (or the last pair); pairs starting at or beyond the workgroup's
    // last slot are not needed
    const long long kend = k0 + S < keff ? k0 + S : keff;
    const long long jlast = k0 + S < keff ? (long long)block_first[blockIdx.x + 1] : nv - 1;
#pragma unroll
    for (int c = 0; c < PT; ++c) {
        const int l = c * kEmitThreads + t;
        const long long j = j0 + l;
        const uint32_t off = j <= jlast ? emit_off[j] : 0xFFFFFFFFu;
        s_off[l] = off;
        s_own[l] = 0u;
        if ((long long)off < kend) {
            const uint32_t q = depth_vals[j];
            const int b = view_of_pair(vt, q);
            const float4* rec = reinterpret_cast<const float4*>(records + (long long)q * kRecFloats);
            const float4 r0 = rec[0], r1 = rec[1], r2 = rec[2];
            const int W = vt.width[b], H = vt.height[b];
            int tx0 = 0, ty0 = 0, tx1 = 0, ty1 = 0;
            tile_rect(r0.x, r0.y, r1.w, r2.x, W, H, vt.tile, tx0, ty0, tx1, ty1);
            s_q[l] = q;
            s_first[l] = (uint32_t)(vt.tile_base[b] + ty0 * vt.ntx[b] + tx0);
            s_wp[l] = (uint32_t)(tx1 - tx0 + 1) | ((uint32_t)vt.ntx[b] << 16);
            s_org[l] = (uint32_t)tx0 | ((uint32_t)ty0 << 16);
            s_wh[l] = (uint32_t)W | ((uint32_t)H << 16);
            s_ell[l] = make_float4(r0.x, r0.y, r0.z, r0.w);
            s_ell2[l] = make_float2(r1.x, tile_tau2(r0.z, r0.w, r1.x, r1.w));
        }
    }
    __syncthreads();
    // slot -> pair: each pair after the first marks its first slot, a prefix maximum fills the
    // rest (every visible pair owns at least one slot, so the marks are distinct)
#pragma unroll
    for (int c = 0; c < PT; ++c) {
        const int l = c * kEmitThreads + t;
        const long long off = (long long)s_off[l];
        if (l > 0 && off < kend) s_own[off - k0] = (uint32_t)l;
    }
    __syncthreads();
    {
        uint32_t v[PT], m = 0;
#pragma unroll
        for (int i = 0; i < PT; ++i) {
            v[i] = max(m, s_own[PT * t + i]);
            m = v[i];
        }
        uint32_t incl = m;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t y = (uint32_t)__shfl_up((int)incl, o, 64);
            if (lane >= o) incl = max(incl, y);
        }
        if (lane == 63) s_wmax[wv] = incl;
        uint32_t excl = (uint32_t)__shfl_up((int)incl, 1, 64);
        if (lane == 0) excl = 0;
        __syncthreads();
#pragma unroll
        for (int x = 0; x < kEmitThreads / 64; ++x)
            if (x < wv) excl = max(excl, s_wmax[x]);
#pragma unroll
        for (int i = 0; i < PT; ++i) s_own[PT * t + i] = max(excl, v[i]);
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < PT; ++c) {
        const long long k = k0 + c * kEmitThreads + t;
        if (k >= keff) break;
        const uint32_t lo = s_own[k - k0];
        const uint32_t r = (uint32_t)(k - (long long)s_off[lo]);
        const uint32_t wp = s_wp[lo], org = s_org[lo], wh = s_wh[lo];
        const uint32_t w = wp & 0xFFFFu;
        // r / w through the float reciprocal: the quotient is at most the rectangle's tile rows
        // (views are under 65,536 pixels a side, so under 2^13 rows), which keeps the float
        // estimate within a hundredth of it, so truncation is off by at most one; the two
        // steps below correct that exactly
        uint32_t row = (uint32_t)((float)r * __builtin_amdgcn_rcpf((float)w));
        row -= row * w > r ? 1u : 0u;
        row += (row + 1u) * w <= r ? 1u : 0u;
        const uint32_t col = r - row * w;
        const int tx = (int)(org & 0xFFFFu) + (int)col;
        const int ty = (int)(org >> 16) + (int)row;
        const float4 e = s_ell[lo];
        const float2 e2 = s_ell2[lo];
        const bool hit = tile_reached(e.x, e.y, e.z, e.w, e2.x, e2.y, tx, ty, vt.tile, (int)(wh & 0xFFFFu),
                                      (int)(wh >> 16));
        tile_keys[k] = hit ? s_first[lo] + row * (wp >> 16) + col : n_tiles;
        tile_vals[k] = s_q[lo];
    }
}

// Tile ranges of the sorted list: four consecutive entries per thread, each compared with
// its neighbours; only entries that open or close a tile's run write.
constexpr int kRangeItems = 4;
__global__ __launch_bounds__(256) void ranges_kernel(const uint32_t* keys, const uint32_t* counters,
                                                     long long n_max, uint32_t n_tiles, uint32_t* ranges) {
    long long n = counters[CNT_LIVE];
    if (n > n_max) n = n_max;
    const long long k0 = ((long long)blockIdx.x * blockDim.x + threadIdx.x) * kRangeItems;
    if (k0 >= n) return;
    uint32_t v[kRangeItems + 2];
    v[0] = k0 > 0 ? keys[k0 - 1] : 0xFFFFFFFFu;
    if (k0 + kRangeItems <= n) {
        const uint4 x = *reinterpret_cast<const uint4*>(keys + k0);  // k0 is a multiple of 4
        v[1] = x.x; v[2] = x.y; v[3] = x.z; v[4] = x.w;
    } else {
#pragma unroll
        for (int j = 0; j < kRangeItems; ++j) v[1 + j] = k0 + j < n ? keys[k0 + j] : 0xFFFFFFFFu;
    }
    v[kRangeItems + 1] = k0 + kRangeItems < n ? keys[k0 + kRangeItems] : 0xFFFFFFFFu;
#pragma unroll
    for (int j = 0; j < kRangeItems; ++j) {
        const long long k = k0 + j;
        const uint32_t t = v[1 + j];
        if (k >= n || t >= n_tiles) continue;
        if (v[j] != t) ranges[2 * (long long)t] = (uint32_t)k;
        if (v[2 + j] != t) ranges[2 * (long long)t + 1] = (uint32_t)(k + 1);
    }
}

// Raster work order (see kWorkStrip): per XCD, its tiles by descending list length in 64
// buckets of 4 log2(length + 1), so the few heavy tiles start early instead of trailing the
// launch, while neighbouring tiles (which share records) stay on one XCD's L2.  Workgroup x
// builds XCD x's list, the slots 8 k + x: it clears them to kNoTile, counts its tiles per
// bucket in LDS, scans the counts in descending bucket order, and lets each tile claim a
// slot of its bucket (the order inside a bucket is that of the claims; any order gives the
// same image).
constexpr int kWorkThreads = 1024, kWorkBuckets = 64;
__global__ __launch_bounds__(kWorkThreads) void work_list_kernel(const uint32_t* ranges, int n_tiles, int n_slots,
                                                                 uint32_t* work) {
    __shared__ uint32_t cnt[kWorkBuckets];
    const int t = threadIdx.x, x = blockIdx.x;
    const int per = n_slots / 8;  // slots of one XCD list (a whole number of strips)
    if (t < kWorkBuckets) cnt[t] = 0;
    for (int k = t; k < per; k += kWorkThreads) work[8 * k + x] = kNoTile;
    __syncthreads();
    // i-th tile of XCD x: strip x + 8 (i / kWorkStrip), position i % kWorkStrip in it
    auto tile_of = [&](int i) { return (x + 8 * (i / kWorkStrip)) * kWorkStrip + i % kWorkStrip; };
    auto bucket = [&](int tile) {
        const uint32_t len = ranges[2 * tile + 1] - ranges[2 * tile];
        const int b = (int)(4.f * log2f((float)len + 1.f));
        return b < kWorkBuckets - 1 ? b : kWorkBuckets - 1;
    };
    for (int i = t; i < per; i += kWorkThreads) {
        const int tile = tile_of(i);
        if (tile < n_tiles) atomicAdd(&cnt[bucket(tile)], 1u);
    }
    __syncthreads();
    if (t == 0) {  // exclusive ranks, largest bucket first
        uint32_t run = 0;
        for (int b = kWorkBuckets - 1; b >= 0; --b) {
            const uint32_t c = cnt[b];
            cnt[b] = run;
            run += c;
        }
    }
    __syncthreads();
    for (int i = t; i < per; i += kWorkThreads) {
        const int tile = tile_of(i);
        if (tile < n_tiles) work[8 * atomicAdd(&cnt[bucket(tile)], 1u) + x] = (uint32_t)tile;
    }
}

// Stage entry from externally supplied records: counts and depth bits per pair.
__global__ void count_from_records_kernel(ViewTable vt, const float* records, const uint8_t* valid,
                                          long long n_pairs, uint32_t* pair_count, uint32_t* pair_z) {
    long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n_pairs) return;
    uint32_t cnt = 0;
    if (valid[q]) {
        const int b = view_of_pair(vt, q);
        const float4* rec = reinterpret_cast<const float4*>(records + q * kRecFloats);
        const float4 r0 = rec[0], r1 = rec[1], r2 = rec[2];
        int tx0, ty0, tx1, ty1;
        if (tile_rect(r0.x, r0.y, r1.w, r2.x, vt.width[b], vt.height[b], vt.tile, tx0, ty0, tx1, ty1))
            cnt = (uint32_t)((tx1 - tx0 + 1) * (ty1 - ty0 + 1));
    }
    pair_count[q] = cnt;
    pair_z[q] = cnt ? __float_as_uint(reinterpret_cast<const float4*>(records + q * kRecFloats)[1].z) : kNoDepth;
}

void launch_count_from_records(const ViewTable& vt, const float* records, const uint8_t* valid,
                               long long n_pairs, uint32_t* pair_count, uint32_t* pair_z,
                               hipStream_t s) {
    if (n_pairs <= 0) return;
    hipLaunchKernelGGL(count_from_records_kernel, dim3((unsigned)((n_pairs + 255) / 256)), dim3(256),
                       0, s, vt, records, valid, n_pairs, pair_count, pair_z);
}

int launch_binning(BinArgs& a, hipStream_t s) {
    const long long Q = a.n_pairs;
    // 1-2. stable depth sort of the visible pairs: the first pass reads every pair's depth
    //    key (pair_z; kNoDepth for a pair no view keeps) with the pair id as value, drops the
    //    invisible ones and counts the visible ones into CNT_V; its last pass also lays out
    //    the pairs' tile counts in depth order, in emit_off
    int r = launch_radix_sort(a.depth_keys, a.depth_vals, Q, nullptr, 32, a.depth_grid, a.sort_tmp, s,
                              a.pair_count, a.emit_off, a.counters + CNT_V, kNoDepth, a.pair_z);
    const uint32_t* dvals = a.depth_vals[r];
    // 3. intersection offsets in depth order (in place), total K, overflow flag, first pair
    //    of each emission workgroup
    launch_emit_scan(a.emit_off, nullptr, a.emit_off, Q, a.counters + CNT_V, a.counters, a.capacity,
                     a.block_first, a.scan_tmp, s);
    // 4. emit (tile id, pair id) in depth order into the buffer from which an even/odd
    //    number of tile-sort passes ends in final_vals
    const int tp = sort_passes(a.tile_bits);
    const int first = (a.final_vals == a.tile_vals[0]) ? (tp % 2) : 1 - (tp % 2);
    const unsigned egrid = (unsigned)((a.capacity + kEmitSlots - 1) / kEmitSlots > 0
                                          ? (a.capacity + kEmitSlots - 1) / kEmitSlots
                                          : 1);
    hipLaunchKernelGGL(emit_kernel, dim3(egrid), dim3(kEmitThreads), 0, s, a.vt, a.records, dvals, a.emit_off,
                       a.block_first, a.counters, a.capacity, a.tile_keys[first], a.tile_vals[first], a.ranges);
    // 5. stable sort by tile id
    uint32_t* tk[2] = {a.tile_keys[first], a.tile_keys[1 - first]};
    uint32_t* tv[2] = {a.tile_vals[first], a.tile_vals[1 - first]};
    //    (its first pass drops the intersections the ellipse test rejected, key n_tiles)
    const long long n_tiles_all = a.vt.tile_base[a.vt.n_views];
    int rt = launch_radix_sort(tk, tv, a.capacity, a.counters + CNT_KEFF, a.tile_bits, a.tile_grid, a.sort_tmp,
                               s, nullptr, nullptr, a.counters + CNT_LIVE, (uint32_t)n_tiles_all);
    // 6. per-tile ranges
    const long long n_tiles = a.vt.tile_base[a.vt.n_views];
    const unsigned rgrid = (unsigned)((a.capacity + 256 * kRangeItems - 1) / (256 * kRangeItems) > 0
                                          ? (a.capacity + 256 * kRangeItems - 1) / (256 * kRangeItems)
                                          : 1);
    hipLaunchKernelGGL(ranges_kernel, dim3(rgrid), dim3(256), 0, s, tk[rt], a.counters, a.capacity,
                       (uint32_t)n_tiles, a.ranges);
    // 7. raster work order
    if (n_tiles > 0)
        hipLaunchKernelGGL(work_list_kernel, dim3(8), dim3(kWorkThreads), 0, s, a.ranges, (int)n_tiles,
                           raster_blocks(a.vt), a.work);
    (void)tv;
    return (int)hipGetLastError();
}

}  // namespace ags
