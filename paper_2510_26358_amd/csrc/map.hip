// Voxel-hashed Gaussian map with a bounded GPU-resident set (Sec. III-B, "Incremental
// Gaussian Mapping": the voxel key equation; "Memory Management": least-recently-used offload
// to host memory above a threshold, reload when a key is met again).  The rules are stated
// with ags_map_insert in agsplat.h.
//
// A key names a group of splats (the one its first point made and that splat's descendants
// by densification); the rules are stated with ags_map_insert and ags_map_lifecycle.
//
// Device state: an open-addressing table (linear probing from the MurmurHash3 64-bit
// finaliser of the key; a slot keeps its key for good) of 64-bit keys and int32 values (the
// group's smallest live id, -1 while the group is empty), with an int32 claim word and an
// int32 hit stamp per slot; per id its key, slot, last_used call and state (offloaded,
// resident, retired).  One insertion call (call number c):
//   1. probe: key per point, find or claim (64-bit CAS) its slot and stamp the slot with c;
//      points of a key absent from the map take the smallest point index on the slot's
//      claim word (atomicMin);
//   2. flag + scan: a point is the first of an absent key when the slot's group is empty and
//      its claim holds the point's index; the scan numbers those keys in point order;
//   3. assign: new ids, slot values, new-splat sources; point ids; a pass over the older ids
//      marks every live id whose slot carries stamp c used, and the offloaded ones for
//      reload; the marks are compacted in id order;
//   4. host: reload rows gathered from the host store through pinned staging;
//   5. if more than tau rows are listed: stable radix sort of the listed rows by last_used,
//      the first (listed - tau) rows are offloaded;
//   6. rebuild: one launch writes the new resident set (packed, row stride = its size) and the
//      offloaded rows (device staging, then pinned host memory; a host thread moves them
//      into the host store while the caller goes on).  When the reloaded or the offloaded rows
//      outnumber the staging rows (max_points), the listed rows go through in chunks of
//      max_points, each staged and copied before the next, on the caller's thread.
#include <limits.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <sys/mman.h>

#include <algorithm>
#include <atomic>
#include <new>
#include <thread>
#include <vector>

#include "common.h"

struct ags_map {
    ags_ctx* ctx;
    ags_map_config cfg;
    int device;
    int F;                         // floats per splat and array (11 + 3 K)
    long long slots;               // table slots (power of two)
    long long list_max;            // max_ids: a listed row is a distinct live id
    long long n_ids;
    long long n_resident;          // rows of the resident set the map returned last
    long long n_offloaded;         // ids in the host store
    int last_frame;
    int seq;                       // insertion calls so far (the slots' hit stamp)
    float ln_s_init, logit_init;
    // device
    unsigned long long* tab_keys;
    int* tab_vals;
    int* tab_claim;
    int* tab_hit;
    unsigned long long* id_key;
    uint32_t* id_slot;
    int* id_last;
    uint8_t* id_res;               // 0 offloaded, 1 resident, 2 retired
    uint32_t* reload_mark;         // [max_ids], zero between calls
    uint32_t* slot;                // [max_points]
    uint32_t* newf;                // [max_points]
    uint32_t* rank;                // [max_points]
    uint32_t* new_point;           // [max_points]
    uint32_t* reload_pos;          // [max_ids]
    uint32_t* reload_list;         // [max_ids]
    uint32_t* keys[2];             // [list_max]
    uint32_t* vals[2];             // [list_max]
    uint32_t* evict_flag;          // [list_max]
    uint32_t* evict_pos;           // [list_max]
    int32_t* evict_ids;            // [max_points], per staging chunk
    uint32_t* counters;            // [4]
    uint32_t* block_sums;
    uint32_t* hist;
    uint32_t* rowtot;
    float* stage_in;               // [max_points][3 F] reloaded rows
    float* stage_out;              // [max_points][3 F] offloaded rows
    // host
    float* pinned;                 // [max_points][3 F]
    float* store;                  // [max_ids][3 F], anonymous mapping, pages committed on use
    size_t store_bytes;
    int32_t* h_evicted;            // [max_points] pinned: ids of the offloaded rows
    std::vector<uint32_t> h_list;  // the reload list, grown as needed
    // offload: the rows leave on a copy stream of the map's own (default priority), so the
    // transfer overlaps the caller's next work; a host thread waits for it and writes the
    // rows into the host store
    hipStream_t cstream;
    hipEvent_t ev_ready, ev_copied;
    std::thread flush;             // host-store writes of the last call's offloaded rows
    std::atomic<int> flush_err;    // a HIP error seen by that thread
};

namespace ags {

constexpr unsigned long long kEmptyKey = ~0ULL;
constexpr uint8_t kOffloaded = 0, kResident = 1, kRetired = 2;
constexpr int kRecompute = -1;                 // hit stamp of a slot whose smallest id was pruned
constexpr float kShC0 = 0.28209479177387814f;  // Y_0^0 = 1 / (2 sqrt(pi))
constexpr int kMapThreads = 256;
constexpr int kMapRows = 16;                   // SH rows per rebuild launch row

struct MapDev {
    unsigned long long* tab_keys;
    int* tab_vals;
    int* tab_claim;
    int* tab_hit;
    unsigned long long mask;
    unsigned long long* id_key;
    uint32_t* id_slot;
    int* id_last;
    uint8_t* id_res;
    uint32_t* reload_mark;
};

struct KeyParams {
    float voxel;
    unsigned long long p1, p2, p3;
};

__device__ __forceinline__ unsigned long long map_key(const float* p, const KeyParams& kp) {
    const long long cx = (long long)floorf(p[0] / kp.voxel);
    const long long cy = (long long)floorf(p[1] / kp.voxel);
    const long long cz = (long long)floorf(p[2] / kp.voxel);
    const unsigned long long k =
        (unsigned long long)cx * kp.p1 + (unsigned long long)cy * kp.p2 + (unsigned long long)cz * kp.p3;
    return k == kEmptyKey ? kEmptyKey - 1 : k;
}

// MurmurHash3's 64-bit finaliser (Appleby): spreads the key's bits over the slot index.
__device__ __forceinline__ unsigned long long fmix64(unsigned long long k) {
    k ^= k >> 33;
    k *= 0xff51afd7ed558ccdULL;
    k ^= k >> 33;
    k *= 0xc4ceb9fe1a85ec53ULL;
    k ^= k >> 33;
    return k;
}

__global__ __launch_bounds__(kMapThreads) void map_probe_kernel(MapDev m, const float* __restrict__ pts,
                                                               long long n, KeyParams kp, int seq, uint32_t* slot) {
    const long long i = (long long)blockIdx.x * kMapThreads + threadIdx.x;
    if (i >= n) return;
    const unsigned long long k = map_key(pts + 3 * i, kp);
    unsigned long long h = fmix64(k) & m.mask;
    // keys only ever change from empty to a key, so a stale empty read is settled by the CAS;
    // the table always has free slots (at most half full), so the walk ends
    for (unsigned long long probe = 0; probe <= m.mask; ++probe) {
        const unsigned long long cur = m.tab_keys[h];
        if (cur == k) break;
        if (cur == kEmptyKey) {
            const unsigned long long old = atomicCAS(&m.tab_keys[h], kEmptyKey, k);
            if (old == kEmptyKey || old == k) break;
        }
        h = (h + 1) & m.mask;
    }
    slot[i] = (uint32_t)h;
    m.tab_hit[h] = seq;
    if (m.tab_vals[h] < 0) atomicMin(&m.tab_claim[h], (int)i);
}

__global__ __launch_bounds__(kMapThreads) void map_flag_kernel(MapDev m, const uint32_t* __restrict__ slot,
                                                              long long n, uint32_t* newf) {
    const long long i = (long long)blockIdx.x * kMapThreads + threadIdx.x;
    if (i >= n) return;
    const uint32_t h = slot[i];
    newf[i] = (m.tab_vals[h] < 0 && m.tab_claim[h] == (int)i) ? 1u : 0u;
}

__global__ __launch_bounds__(kMapThreads) void map_assign_kernel(MapDev m, long long n,
                                                                const uint32_t* __restrict__ slot,
                                                                const uint32_t* __restrict__ newf,
                                                                const uint32_t* __restrict__ rank, int id_base,
                                                                int frame, uint32_t* new_point) {
    const long long i = (long long)blockIdx.x * kMapThreads + threadIdx.x;
    if (i >= n || !newf[i]) return;
    const uint32_t h = slot[i];
    const uint32_t r = rank[i];
    const int id = id_base + (int)r;
    m.tab_vals[h] = id;
    m.tab_claim[h] = INT_MAX;
    m.id_key[id] = m.tab_keys[h];
    m.id_slot[id] = h;
    m.id_last[id] = frame;
    m.id_res[id] = kResident;
    new_point[r] = (uint32_t)i;
}

// A point's id: its group's smallest live id (the new id for a key the call made).
__global__ __launch_bounds__(kMapThreads) void map_point_id_kernel(MapDev m, long long n,
                                                                  const uint32_t* __restrict__ slot,
                                                                  int32_t* point_id) {
    const long long i = (long long)blockIdx.x * kMapThreads + threadIdx.x;
    if (i < n) point_id[i] = m.tab_vals[slot[i]];
}

// Ids older than the call: a live id whose slot the call stamped is used now, and reloaded
// if it was offloaded.
__global__ __launch_bounds__(kMapThreads) void map_hit_kernel(MapDev m, long long n_old, int seq, int frame) {
    const long long id = (long long)blockIdx.x * kMapThreads + threadIdx.x;
    if (id >= n_old) return;
    const uint8_t st = m.id_res[id];
    const bool hit = st != kRetired && m.tab_hit[m.id_slot[id]] == seq;
    if (hit) m.id_last[id] = frame;
    m.reload_mark[id] = hit && st == kOffloaded ? 1u : 0u;
}

// Offloaded ids met by the call, in id order; they become resident.
__global__ __launch_bounds__(kMapThreads) void map_reload_list_kernel(MapDev m, long long n_ids,
                                                                     const uint32_t* __restrict__ pos,
                                                                     uint32_t* list) {
    const long long id = (long long)blockIdx.x * kMapThreads + threadIdx.x;
    if (id >= n_ids || !m.reload_mark[id]) return;
    list[pos[id]] = (uint32_t)id;
    m.reload_mark[id] = 0u;
    m.id_res[id] = kResident;
}

struct ListArgs {
    long long n_in, n_new, n_list;
    int id_base;
    const int32_t* in_ids;
    const uint32_t* reload_list;
};

__device__ __forceinline__ int list_id(const ListArgs& l, long long q) {
    if (q < l.n_in) return l.in_ids[q];
    if (q < l.n_in + l.n_new) return l.id_base + (int)(q - l.n_in);
    return (int)l.reload_list[q - l.n_in - l.n_new];
}

__global__ __launch_bounds__(kMapThreads) void map_lru_keys_kernel(MapDev m, ListArgs l, uint32_t* keys,
                                                                  uint32_t* vals) {
    const long long q = (long long)blockIdx.x * kMapThreads + threadIdx.x;
    if (q >= l.n_list) return;
    keys[q] = (uint32_t)m.id_last[list_id(l, q)];
    vals[q] = (uint32_t)q;
}

__global__ __launch_bounds__(kMapThreads) void map_mark_evict_kernel(const uint32_t* __restrict__ sorted_rows,
                                                                    long long n_evict, uint32_t* flag) {
    const long long e = (long long)blockIdx.x * kMapThreads + threadIdx.x;
    if (e < n_evict) flag[sorted_rows[e]] = 1u;
}

struct RebuildArgs {
    ListArgs l;
    int F, k3, chunks;
    long long n_keep;
    long long q_begin, q_end;       // the listed rows this launch moves
    long long reload_off;           // reload rank of stage_in's first row
    long long evict_off;            // offload rank of stage_out's (and evict_ids') first row
    const float* in[3][5];
    float* out[3][5];
    const float* pts;
    const float* cols;
    const uint32_t* new_point;
    const float* stage_in;          // reloaded rows [r - reload_off][3 F]
    float* stage_out;               // offloaded rows [e - evict_off][3 F]
    const uint32_t* evict_flag;     // null: nothing offloaded
    const uint32_t* evict_pos;
    int32_t* out_ids;
    int32_t* evict_ids;             // map-owned [max_points], indexed e - evict_off
    int32_t* evict_ids_user;        // or null, indexed e
    float ln_s_init, logit_init;
};

// Row offsets of the five fields inside one splat's F floats.
__device__ __forceinline__ int field_base(int f) { return f == 0 ? 0 : f == 1 ? 3 : f == 2 ? 6 : f == 3 ? 10 : 11; }

// Value of row r (of F) of a new splat's parameters made from point i.
__device__ __forceinline__ float new_value(const RebuildArgs& a, long long i, int r) {
    if (r < 3) return a.pts[3 * i + r];
    if (r < 6) return a.ln_s_init;
    if (r < 10) return r == 6 ? 1.f : 0.f;
    if (r == 10) return a.logit_init;
    const int s = r - 11;                       // SH row: coefficient s / 3, channel s % 3
    return s < 3 ? (a.cols[3 * i + s] - 0.5f) / kShC0 : 0.f;
}

// Moves `rows` rows (row strides sn in, dn out) of one field from column q to column d.
template <int R>
__device__ __forceinline__ void map_move(const float* __restrict__ src, long long sn, float* __restrict__ dst,
                                         long long dn, int rows, long long q, long long d) {
    float v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) v[r] = src[(long long)(r < rows ? r : rows - 1) * sn + q];
#pragma unroll
    for (int r = 0; r < R; ++r)
        if (r < rows) dst[(long long)r * dn + d] = v[r];
}

// grid (ceil((q_end - q_begin) / 256), 3 * chunks): a thread moves rows [r0, r0 + rows) of
// one array (parameters, m, v) of listed row q to its new place.  Chunk 0 = the 11 rows of
// means, log-scales, quaternion and logit (and the row's id bookkeeping); chunks 1.. = SH
// rows in groups of kMapRows.
__global__ __launch_bounds__(kMapThreads) void map_rebuild_kernel(RebuildArgs a, MapDev m) {
    const long long q = a.q_begin + (long long)blockIdx.x * kMapThreads + threadIdx.x;
    if (q >= a.q_end) return;
    const int t = blockIdx.y / a.chunks, c = blockIdx.y % a.chunks;
    const bool evict = a.evict_flag && a.evict_flag[q];
    const long long ep = a.evict_flag ? (long long)a.evict_pos[q] : 0;
    const long long es = ep - a.evict_off;      // staging row of an offloaded row
    const long long dst = q - ep;               // row in the new resident set
    const int r0 = c == 0 ? 0 : 11 + (c - 1) * kMapRows;
    const int rows = c == 0 ? 11 : (a.k3 - (c - 1) * kMapRows < kMapRows ? a.k3 - (c - 1) * kMapRows : kMapRows);
    const int kind = q < a.l.n_in ? 0 : (q < a.l.n_in + a.l.n_new ? 1 : 2);
    if (t == 0 && c == 0) {
        const int id = list_id(a.l, q);
        if (evict) {
            m.id_res[id] = kOffloaded;
            a.evict_ids[es] = id;
            if (a.evict_ids_user) a.evict_ids_user[ep] = id;
        } else {
            a.out_ids[dst] = id;
        }
    }
    if (kind == 0 && !evict) {
        // a kept row of the previous set: SoA to SoA, all loads before the stores
        if (c == 0) {
            const int fr[4] = {3, 3, 4, 1};
#pragma unroll
            for (int f = 0; f < 4; ++f)
                map_move<4>(a.in[t][f], a.l.n_in, a.out[t][f], a.n_keep, fr[f], q, dst);
        } else {
            const long long s0 = (long long)(c - 1) * kMapRows;
            map_move<kMapRows>(a.in[t][4] + s0 * a.l.n_in, a.l.n_in, a.out[t][4] + s0 * a.n_keep, a.n_keep, rows, q,
                               dst);
        }
        return;
    }
    float v[kMapRows];
#pragma unroll
    for (int k = 0; k < kMapRows; ++k) {
        const int r = r0 + (k < rows ? k : rows - 1);
        float x;
        if (kind == 0) {
            int f = r < 3 ? 0 : r < 6 ? 1 : r < 10 ? 2 : r < 11 ? 3 : 4;
            x = a.in[t][f][(long long)(r - field_base(f)) * a.l.n_in + q];
        } else if (kind == 1) {
            x = t == 0 ? new_value(a, a.new_point[q - a.l.n_in], r) : 0.f;
        } else {
            x = a.stage_in[(q - a.l.n_in - a.l.n_new - a.reload_off) * 3 * a.F + (long long)t * a.F + r];
        }
        v[k] = x;
    }
    if (evict) {
        float* row = a.stage_out + es * 3 * a.F + (long long)t * a.F;
#pragma unroll
        for (int k = 0; k < kMapRows; ++k)
            if (k < rows) row[r0 + k] = v[k];
    } else {
#pragma unroll
        for (int k = 0; k < kMapRows; ++k) {
            if (k < rows) {
                const int r = r0 + k;
                const int f = r < 3 ? 0 : r < 6 ? 1 : r < 10 ? 2 : r < 11 ? 3 : 4;
                a.out[t][f][(long long)(r - field_base(f)) * a.n_keep + dst] = v[k];
            }
        }
    }
}

// ---- the map's side of a lifecycle pass over the resident set (ags_map_lifecycle)

struct LifeArgs {
    const int32_t* ids;             // [n] resident ids, row order
    const uint8_t* actions;         // [n] 0 keep, 1 prune, 2 duplicate, 3 split
    long long n, n_ids;
    uint32_t* outs;                 // [n] output rows of each input
    uint32_t* extra;                // [n] 1 for a duplicated or split input
    uint32_t* out_pos;              // [n] exclusive scan of outs
    uint32_t* new_rank;             // [n] exclusive scan of extra
    uint32_t* bad;                  // counter: refused inputs
};

// Whether a row's id is refused: out of range, not resident, or seen before in the same list
// (each id is counted on reload_mark, zero between calls; map_ids_unmark_kernel clears it).
__device__ __forceinline__ bool id_refused(const MapDev& m, int id, long long n_ids) {
    if (id < 0 || (long long)id >= n_ids) return true;
    return m.id_res[id] != kResident || atomicAdd(&m.reload_mark[id], 1u) != 0u;
}

// The resident ids an insertion call is given: refused ones are counted.
__global__ __launch_bounds__(kMapThreads) void map_ids_check_kernel(MapDev m, const int32_t* __restrict__ ids,
                                                                   long long n, long long n_ids, uint32_t* bad) {
    const long long q = (long long)blockIdx.x * kMapThreads + threadIdx.x;
    if (q < n && id_refused(m, ids[q], n_ids)) atomicAdd(bad, 1u);
}

__global__ __launch_bounds__(kMapThreads) void map_ids_unmark_kernel(MapDev m, const int32_t* __restrict__ ids,
                                                                    long long n, long long n_ids) {
    const long long q = (long long)blockIdx.x * kMapThreads + threadIdx.x;
    if (q >= n) return;
    const int id = ids[q];
    if (id >= 0 && (long long)id < n_ids) m.reload_mark[id] = 0u;
}

// Validation and output counts of a lifecycle pass's rows.
__global__ __launch_bounds__(kMapThreads) void map_life_count_kernel(LifeArgs a, MapDev m) {
    const long long q = (long long)blockIdx.x * kMapThreads + threadIdx.x;
    if (q >= a.n) return;
    const unsigned act = a.actions[q];
    const bool bad = id_refused(m, a.ids[q], a.n_ids) || act > 3u;
    if (bad) atomicAdd(a.bad, 1u);
    const bool two = !bad && act >= 2u;
    a.outs[q] = bad || act == 1u ? 0u : (two ? 2u : 1u);
    a.extra[q] = two ? 1u : 0u;
}

// Output ids, new ids (the parent's key, slot and last use) and retirements.  A pruned id
// that is its group's smallest sets the slot's value to INT_MAX and stamps the slot for the
// recomputation that follows.
__global__ __launch_bounds__(kMapThreads) void map_life_apply_kernel(LifeArgs a, MapDev m, int32_t* out_ids) {
    const long long q = (long long)blockIdx.x * kMapThreads + threadIdx.x;
    if (q >= a.n) return;
    const int id = a.ids[q];
    const unsigned act = a.actions[q];
    if (act == 1u) {
        m.id_res[id] = kRetired;
        const uint32_t h = m.id_slot[id];
        if (m.tab_vals[h] == id) {
            m.tab_vals[h] = INT_MAX;
            m.tab_hit[h] = kRecompute;
        }
        return;
    }
    const long long p = a.out_pos[q];
    out_ids[p] = id;
    if (act >= 2u) {
        const int c = (int)(a.n_ids + a.new_rank[q]);
        out_ids[p + 1] = c;
        m.id_key[c] = m.id_key[id];
        m.id_slot[c] = m.id_slot[id];
        m.id_last[c] = m.id_last[id];
        m.id_res[c] = kResident;
    }
}

// The smallest live id of every group whose smallest was pruned.
__global__ __launch_bounds__(kMapThreads) void map_life_min_kernel(MapDev m, long long n_ids) {
    const long long id = (long long)blockIdx.x * kMapThreads + threadIdx.x;
    if (id >= n_ids || m.id_res[id] == kRetired) return;
    const uint32_t h = m.id_slot[id];
    if (m.tab_hit[h] == kRecompute) atomicMin(&m.tab_vals[h], (int)id);
}

struct PackArgs {
    const float* in[3][5];          // the pass's output rows, row stride sn
    float* out[3][5];               // the resident set, row stride dn (= its size)
    long long sn, dn;
    int k3, chunks;
};

// grid (ceil(dn / 256), 3 * chunks): row p of one array (parameters, m, v), chunk 0 = means,
// log-scales, quaternion and logit, chunks 1.. = SH rows in groups of kMapRows.
__global__ __launch_bounds__(kMapThreads) void map_life_pack_kernel(PackArgs a) {
    const long long p = (long long)blockIdx.x * kMapThreads + threadIdx.x;
    if (p >= a.dn) return;
    const int t = blockIdx.y / a.chunks, c = blockIdx.y % a.chunks;
    if (c == 0) {
        const int fr[4] = {3, 3, 4, 1};
#pragma unroll
        for (int f = 0; f < 4; ++f) map_move<4>(a.in[t][f], a.sn, a.out[t][f], a.dn, fr[f], p, p);
    } else {
        const long long s0 = (long long)(c - 1) * kMapRows;
        const int rows = a.k3 - (int)s0 < kMapRows ? a.k3 - (int)s0 : kMapRows;
        map_move<kMapRows>(a.in[t][4] + s0 * a.sn, a.sn, a.out[t][4] + s0 * a.dn, a.dn, rows, p, p);
    }
}

// Groups left without a live id: the key is absent from the map again (value -1; the claim
// word is INT_MAX since the slot was assigned).  Clears the recomputation stamps.
__global__ __launch_bounds__(kMapThreads) void map_life_settle_kernel(LifeArgs a, MapDev m) {
    const long long q = (long long)blockIdx.x * kMapThreads + threadIdx.x;
    if (q >= a.n || a.actions[q] != 1u) return;
    const uint32_t h = m.id_slot[a.ids[q]];
    if (m.tab_hit[h] == kRecompute) {
        if (m.tab_vals[h] == INT_MAX) m.tab_vals[h] = -1;
        m.tab_hit[h] = 0;
    }
}

}  // namespace ags

using namespace ags;

namespace {

constexpr size_t kMapAlign = 256;
size_t map_align(size_t x) { return (x + kMapAlign - 1) / kMapAlign * kMapAlign; }

bool map_gaussians_ok(const ags_gaussians* g, int deg) {
    if (!g || g->n < 0 || g->sh_degree != deg) return false;
    if (g->n > 0 && (!g->means || !g->log_scales || !g->quats || !g->opacity_logits || !g->sh)) return false;
    return true;
}

unsigned grid_of(long long n) { return (unsigned)((n + kMapThreads - 1) / kMapThreads); }

MapDev dev_of(const ags_map* mp) {
    MapDev m;
    m.tab_keys = mp->tab_keys;
    m.tab_vals = mp->tab_vals;
    m.tab_claim = mp->tab_claim;
    m.tab_hit = mp->tab_hit;
    m.mask = (unsigned long long)(mp->slots - 1);
    m.id_key = mp->id_key;
    m.id_slot = mp->id_slot;
    m.id_last = mp->id_last;
    m.id_res = mp->id_res;
    m.reload_mark = mp->reload_mark;
    return m;
}

// Runs fn(begin, end) over [0, n) split across up to 16 host threads (one when n is small).
template <class Fn>
void parallel_rows(long long n, long long min_per_thread, Fn fn) {
    const unsigned hw = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    const long long t = std::max(1LL, std::min<long long>(hw, n / std::max(1LL, min_per_thread)));
    std::vector<std::thread> pool;
    long long done = 0;  // rows [0, done) handed to threads; the rest run on this thread
    try {
        pool.reserve((size_t)t);
        for (long long k = 1; k < t; ++k) {
            pool.emplace_back(fn, n * k / t, n * (k + 1) / t);
            done = n * (k + 1) / t;
        }
    } catch (...) {
    }
    fn(0LL, t > 1 ? n / t : n);
    if (t > 1 && done < n) fn(pool.empty() ? n / t : done, n);
    for (auto& th : pool) th.join();
}

// Waits for the host-store writes of the previous call (they read the pinned staging);
// AGS_ERR_HIP if its copy failed.
int flush_join(ags_map* m) {
    if (m->flush.joinable()) m->flush.join();
    return m->flush_err.exchange(0) ? AGS_ERR_HIP : AGS_OK;
}

void map_free(ags_map* m) {
    (void)flush_join(m);
    void* dev[] = {m->tab_keys, m->tab_vals, m->tab_claim, m->tab_hit, m->id_key, m->id_slot, m->id_last,
                   m->id_res, m->reload_mark,
                   m->slot, m->newf, m->rank, m->new_point, m->reload_pos, m->reload_list, m->keys[0],
                   m->keys[1], m->vals[0], m->vals[1], m->evict_flag, m->evict_pos, m->evict_ids,
                   m->counters, m->block_sums, m->hist, m->rowtot, m->stage_in, m->stage_out};
    for (void* p : dev)
        if (p) (void)hipFree(p);
    if (m->pinned) (void)hipHostFree(m->pinned);
    if (m->h_evicted) (void)hipHostFree(m->h_evicted);
    if (m->ev_ready) (void)hipEventDestroy(m->ev_ready);
    if (m->ev_copied) (void)hipEventDestroy(m->ev_copied);
    if (m->cstream) (void)hipStreamDestroy(m->cstream);
    if (m->store) munmap(m->store, m->store_bytes);
    delete m;
}

__global__ void map_fill_u64_kernel(unsigned long long* p, unsigned long long v, long long n) {
    const long long i = (long long)blockIdx.x * kMapThreads + threadIdx.x;
    if (i < n) p[i] = v;
}

}  // namespace

extern "C" {

int ags_map_config_default(ags_map_config* c) {
    if (!c) return AGS_ERR_INVALID_ARG;
    c->voxel = 0.05f;
    c->s_init = 0.005f;
    c->o_init = 0.1f;
    c->sh_degree = 3;
    c->prime[0] = 73856093ULL;
    c->prime[1] = 19349663ULL;
    c->prime[2] = 83492791ULL;
    c->max_ids = 1LL << 22;
    c->max_points = 1LL << 20;
    c->tau = 1LL << 20;
    return AGS_OK;
}

int ags_map_create(ags_ctx* ctx, const ags_map_config* cfg, ags_map** out) {
    if (!ctx || !cfg || !out) return AGS_ERR_INVALID_ARG;
    *out = nullptr;
    if (!(cfg->voxel > 0.f) || !(cfg->s_init > 0.f) || !(cfg->o_init > 0.f && cfg->o_init < 1.f))
        return AGS_ERR_INVALID_ARG;
    if (cfg->sh_degree < 0 || cfg->sh_degree > 3) return AGS_ERR_INVALID_ARG;
    if (cfg->max_ids < 1 || cfg->max_ids > (1LL << 30) || cfg->max_points < 1 || cfg->max_points > (1LL << 28) ||
        cfg->tau < 1 || cfg->tau > (1LL << 30))
        return AGS_ERR_INVALID_ARG;
    ags_map* m = new (std::nothrow) ags_map();
    if (!m) return AGS_ERR_INVALID_ARG;
    memset(m->keys, 0, sizeof(m->keys));
    memset(m->vals, 0, sizeof(m->vals));
    m->ctx = ctx;
    m->cfg = *cfg;
    m->device = ctx_device(ctx);
    const int K = (cfg->sh_degree + 1) * (cfg->sh_degree + 1);
    m->F = 11 + 3 * K;
    long long slots = 1;
    while (slots < 2 * cfg->max_ids) slots <<= 1;
    m->slots = slots;
    m->list_max = cfg->max_ids;
    m->n_ids = 0;
    m->n_resident = 0;
    m->n_offloaded = 0;
    m->last_frame = -1;
    m->seq = 0;
    m->ln_s_init = (float)log((double)cfg->s_init);
    m->logit_init = (float)log((double)cfg->o_init / (1.0 - (double)cfg->o_init));
    if (hipSetDevice(m->device) != hipSuccess) {
        int rc = ctx_record_hip(ctx, hipGetLastError());
        delete m;
        return rc;
    }
    const long long P = cfg->max_points, I = cfg->max_ids, Lm = m->list_max;
    const size_t row_bytes = (size_t)3 * m->F * sizeof(float);
    const int grid = sort_grid(Lm);
    long long nb = scan_blocks(Lm > I ? Lm : I);
    if (nb < 1) nb = 1;
    struct A {
        void** p;
        size_t bytes;
    } allocs[] = {
        {(void**)&m->tab_keys, 8 * (size_t)slots}, {(void**)&m->tab_vals, 4 * (size_t)slots},
        {(void**)&m->tab_claim, 4 * (size_t)slots}, {(void**)&m->tab_hit, 4 * (size_t)slots},
        {(void**)&m->id_key, 8 * (size_t)I}, {(void**)&m->id_slot, 4 * (size_t)I},
        {(void**)&m->id_last, 4 * (size_t)I}, {(void**)&m->id_res, (size_t)I},
        {(void**)&m->reload_mark, 4 * (size_t)I}, {(void**)&m->slot, 4 * (size_t)P},
        {(void**)&m->newf, 4 * (size_t)P}, {(void**)&m->rank, 4 * (size_t)P},
        {(void**)&m->new_point, 4 * (size_t)P}, {(void**)&m->reload_pos, 4 * (size_t)I},
        {(void**)&m->reload_list, 4 * (size_t)I}, {(void**)&m->keys[0], 4 * (size_t)Lm},
        {(void**)&m->keys[1], 4 * (size_t)Lm}, {(void**)&m->vals[0], 4 * (size_t)Lm},
        {(void**)&m->vals[1], 4 * (size_t)Lm}, {(void**)&m->evict_flag, 4 * (size_t)Lm},
        {(void**)&m->evict_pos, 4 * (size_t)Lm}, {(void**)&m->evict_ids, 4 * (size_t)P},
        {(void**)&m->counters, 16}, {(void**)&m->block_sums, 4 * (size_t)nb},
        {(void**)&m->hist, 4 * (size_t)sort_hist_entries(grid)}, {(void**)&m->rowtot, 4 * (size_t)sort_rowtot_entries()},
        {(void**)&m->stage_in, row_bytes * (size_t)P}, {(void**)&m->stage_out, row_bytes * (size_t)P},
    };
    for (auto& a : allocs) {
        if (hipMalloc(a.p, map_align(a.bytes)) != hipSuccess) {
            int rc = ctx_record_hip(ctx, hipGetLastError());
            map_free(m);
            return rc;
        }
    }
    if (hipHostMalloc((void**)&m->pinned, row_bytes * (size_t)P, hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void**)&m->h_evicted, 4 * (size_t)P, hipHostMallocDefault) != hipSuccess ||
        hipStreamCreateWithFlags(&m->cstream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&m->ev_ready, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&m->ev_copied, hipEventDisableTiming) != hipSuccess) {
        int rc = ctx_record_hip(ctx, hipGetLastError());
        map_free(m);
        return rc;
    }
    // host store: reserved, committed page by page as rows are offloaded (transparent huge
    // pages where the system allows them, so that committing costs few faults)
    m->store_bytes = row_bytes * (size_t)I;
    void* st = mmap(nullptr, m->store_bytes, PROT_READ | PROT_WRITE, MAP_PRIVATE | MAP_ANONYMOUS | MAP_NORESERVE,
                    -1, 0);
    if (st == MAP_FAILED) {
        map_free(m);
        return AGS_ERR_INVALID_ARG;
    }
    (void)madvise(st, m->store_bytes, MADV_HUGEPAGE);
    m->store = (float*)st;
    hipStream_t s = nullptr;
    hipLaunchKernelGGL(map_fill_u64_kernel, dim3(grid_of(slots)), dim3(kMapThreads), 0, s, m->tab_keys, kEmptyKey,
                       slots);
    launch_fill_u32(reinterpret_cast<uint32_t*>(m->tab_vals), 0xffffffffu, slots, s);
    launch_fill_u32(reinterpret_cast<uint32_t*>(m->tab_claim), (uint32_t)INT_MAX, slots, s);
    launch_fill_u32(reinterpret_cast<uint32_t*>(m->tab_hit), 0u, slots, s);
    launch_fill_u32(m->reload_mark, 0u, I, s);
    launch_fill_u32(reinterpret_cast<uint32_t*>(m->id_last), 0u, I, s);
    if (hipMemsetAsync(m->id_res, 0, (size_t)I, s) != hipSuccess || hipStreamSynchronize(s) != hipSuccess) {
        int rc = ctx_record_hip(ctx, hipGetLastError());
        map_free(m);
        return rc;
    }
    *out = m;
    return AGS_OK;
}

int ags_map_destroy(ags_map* map) {
    if (!map) return AGS_ERR_INVALID_ARG;
    (void)hipSetDevice(map->device);
    (void)hipDeviceSynchronize();
    map_free(map);
    return AGS_OK;
}

int ags_map_insert(ags_map* mp, const float* points, const float* colors, int64_t n_points, int32_t frame,
                   const ags_gaussians* in, const ags_gaussians* in_m, const ags_gaussians* in_v,
                   const int32_t* in_ids, ags_gaussians* out, ags_gaussians* out_m, ags_gaussians* out_v,
                   int32_t* out_ids, int32_t* point_id, int32_t* evicted_ids, ags_map_counts* counts,
                   void* stream) {
    if (!mp || !counts) return AGS_ERR_INVALID_ARG;
    const ags_map_config& cfg = mp->cfg;
    const int deg = cfg.sh_degree;
    if (n_points < 0 || n_points > cfg.max_points || (n_points > 0 && (!points || !colors))) return AGS_ERR_INVALID_ARG;
    if (frame < 0 || frame < mp->last_frame) return AGS_ERR_INVALID_ARG;
    if (!map_gaussians_ok(in, deg) || !map_gaussians_ok(in_m, deg) || !map_gaussians_ok(in_v, deg) ||
        !map_gaussians_ok(out, deg) || !map_gaussians_ok(out_m, deg) || !map_gaussians_ok(out_v, deg))
        return AGS_ERR_INVALID_ARG;
    const long long n_in = in->n;
    if (in_m->n != n_in || in_v->n != n_in || n_in != mp->n_resident || (n_in > 0 && !in_ids))
        return AGS_ERR_INVALID_ARG;
    if (out_m->n != out->n || out_v->n != out->n || !out_ids) return AGS_ERR_INVALID_ARG;
    const long long most = n_in + n_points + mp->n_offloaded;  // listed rows at most
    const long long need = most < cfg.tau ? most : cfg.tau;
    if (out->n < need) return AGS_ERR_INVALID_ARG;
    if (mp->n_ids + n_points > cfg.max_ids) return AGS_ERR_CAPACITY;
    ags_ctx* ctx = mp->ctx;
    if (hipSetDevice(mp->device) != hipSuccess) return ctx_record_hip(ctx, hipGetLastError());
    if (flush_join(mp) != AGS_OK) return AGS_ERR_HIP;  // the previous call's offload failed
    hipStream_t s = (hipStream_t)stream;
    const MapDev m = dev_of(mp);
    KeyParams kp;
    kp.voxel = cfg.voxel;
    kp.p1 = cfg.prime[0];
    kp.p2 = cfg.prime[1];
    kp.p3 = cfg.prime[2];
    const int id_base = (int)mp->n_ids;
    ScanTemp st;
    st.block_sums = mp->block_sums;
    // the rows' ids: every one resident, none twice (nothing changes otherwise)
    if (n_in > 0) {
        uint32_t bad = 0;
        launch_fill_u32(mp->counters + 3, 0u, 1, s);
        hipLaunchKernelGGL(map_ids_check_kernel, dim3(grid_of(n_in)), dim3(kMapThreads), 0, s, m, in_ids, n_in,
                           (long long)id_base, mp->counters + 3);
        hipLaunchKernelGGL(map_ids_unmark_kernel, dim3(grid_of(n_in)), dim3(kMapThreads), 0, s, m, in_ids, n_in,
                           (long long)id_base);
        if (hipMemcpyAsync(&bad, mp->counters + 3, 4, hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            return ctx_record_hip(ctx, hipGetLastError());
        if (bad != 0) return AGS_ERR_INVALID_ARG;
    }
    const int seq = ++mp->seq;
    // 1-3: probe, first points of absent keys, ids, hits and reload marks
    {
    StageTimer tm(ctx, ST_MAP_PROBE, s);
    launch_fill_u32(mp->counters, 0u, 4, s);
    if (n_points > 0) {
        const unsigned g = grid_of(n_points);
        hipLaunchKernelGGL(map_probe_kernel, dim3(g), dim3(kMapThreads), 0, s, m, points, (long long)n_points, kp,
                           seq, mp->slot);
        hipLaunchKernelGGL(map_flag_kernel, dim3(g), dim3(kMapThreads), 0, s, m, mp->slot, (long long)n_points,
                           mp->newf);
        launch_scan(mp->newf, nullptr, false, mp->rank, n_points, nullptr, mp->counters, st, s);
        hipLaunchKernelGGL(map_assign_kernel, dim3(g), dim3(kMapThreads), 0, s, m, (long long)n_points, mp->slot,
                           mp->newf, mp->rank, id_base, (int)frame, mp->new_point);
        if (point_id)
            hipLaunchKernelGGL(map_point_id_kernel, dim3(g), dim3(kMapThreads), 0, s, m, (long long)n_points,
                               mp->slot, point_id);
        if (id_base > 0) {
            hipLaunchKernelGGL(map_hit_kernel, dim3(grid_of(id_base)), dim3(kMapThreads), 0, s, m,
                               (long long)id_base, seq, (int)frame);
            launch_scan(mp->reload_mark, nullptr, true, mp->reload_pos, id_base, nullptr, mp->counters + 1, st, s);
            hipLaunchKernelGGL(map_reload_list_kernel, dim3(grid_of(id_base)), dim3(kMapThreads), 0, s, m,
                               (long long)id_base, mp->reload_pos, mp->reload_list);
        }
    }
    }
    uint32_t hc[4];
    if (hipMemcpyAsync(hc, mp->counters, sizeof(hc), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return ctx_record_hip(ctx, hipGetLastError());
    const long long n_new = hc[0], n_reload = hc[1];
    const size_t row_f = (size_t)3 * mp->F;
    const long long S = cfg.max_points;          // staging rows
    if (n_reload > 0) {
        if ((long long)mp->h_list.size() < n_reload) {
            try {
                mp->h_list.resize((size_t)n_reload);
            } catch (...) {
                return AGS_ERR_HIP;   // the map's state is undefined, as after any failed call
            }
        }
        if (hipMemcpyAsync(mp->h_list.data(), mp->reload_list, 4 * (size_t)n_reload, hipMemcpyDeviceToHost, s) !=
                hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            return ctx_record_hip(ctx, hipGetLastError());
    }
    ListArgs l;
    l.n_in = n_in;
    l.n_new = n_new;
    l.n_list = n_in + n_new + n_reload;
    l.id_base = id_base;
    l.in_ids = in_ids;
    l.reload_list = mp->reload_list;
    // listed ids are distinct live ids, so n_list <= max_ids (the list buffers' size)
    if (l.n_list > mp->list_max) return AGS_ERR_CAPACITY;
    const long long n_keep = l.n_list < cfg.tau ? l.n_list : cfg.tau;
    const long long n_evict = l.n_list - n_keep;
    const bool chunked = n_reload > S || n_evict > S;
    // host-store rows [r0, r1) of the reload list into stage_in, through pinned memory
    auto stage_reloads = [&](long long r0, long long r1) -> int {
        if (r1 <= r0) return AGS_OK;
        parallel_rows(r1 - r0, 2048, [&](long long b, long long e) {
            for (long long r = b; r < e; ++r)
                memcpy(mp->pinned + r * row_f, mp->store + (size_t)mp->h_list[r0 + r] * row_f, row_f * sizeof(float));
        });
        StageTimer tm(ctx, ST_MAP_COPY, s);
        if (hipMemcpyAsync(mp->stage_in, mp->pinned, row_f * sizeof(float) * (size_t)(r1 - r0), hipMemcpyHostToDevice,
                           s) != hipSuccess)
            return ctx_record_hip(ctx, hipGetLastError());
        return AGS_OK;
    };
    // 4: reloaded rows from the host store (all of them, unless they go in chunks)
    if (!chunked) {
        const int rc = stage_reloads(0, n_reload);
        if (rc != AGS_OK) return rc;
    }
    // 5: least recently used rows beyond tau
    if (n_evict > 0) {
        StageTimer tm(ctx, ST_MAP_LRU, s);
        const unsigned g = grid_of(l.n_list);
        hipLaunchKernelGGL(map_lru_keys_kernel, dim3(g), dim3(kMapThreads), 0, s, m, l, mp->keys[0], mp->vals[0]);
        int bits = 0;
        while (bits < 31 && (frame >> bits) != 0) ++bits;
        SortTemp sort_tmp;
        sort_tmp.hist = mp->hist;
        sort_tmp.rowtot = mp->rowtot;
        const int r = launch_radix_sort(mp->keys, mp->vals, l.n_list, nullptr, bits, sort_grid(l.n_list), sort_tmp, s);
        launch_fill_u32(mp->evict_flag, 0u, l.n_list, s);
        hipLaunchKernelGGL(map_mark_evict_kernel, dim3(grid_of(n_evict)), dim3(kMapThreads), 0, s, mp->vals[r],
                           n_evict, mp->evict_flag);
        launch_scan(mp->evict_flag, nullptr, false, mp->evict_pos, l.n_list, nullptr, nullptr, st, s);
    }
    // 6: the new resident set and the offloaded rows
    RebuildArgs a;
    memset(&a, 0, sizeof(a));
    a.l = l;
    a.F = mp->F;
    a.k3 = 3 * (deg + 1) * (deg + 1);
    a.chunks = 1 + (a.k3 + kMapRows - 1) / kMapRows;
    a.n_keep = n_keep;
    {
        const ags_gaussians* ins[3] = {in, in_m, in_v};
        ags_gaussians* outs[3] = {out, out_m, out_v};
        for (int t = 0; t < 3; ++t) {
            const float* src[5] = {ins[t]->means, ins[t]->log_scales, ins[t]->quats, ins[t]->opacity_logits,
                                   ins[t]->sh};
            float* dst[5] = {outs[t]->means, outs[t]->log_scales, outs[t]->quats, outs[t]->opacity_logits,
                             outs[t]->sh};
            for (int f = 0; f < 5; ++f) {
                a.in[t][f] = src[f];
                a.out[t][f] = dst[f];
            }
        }
    }
    a.pts = points;
    a.cols = colors;
    a.new_point = mp->new_point;
    a.stage_in = mp->stage_in;
    a.stage_out = mp->stage_out;
    a.evict_flag = n_evict > 0 ? mp->evict_flag : nullptr;
    a.evict_pos = mp->evict_pos;
    a.out_ids = out_ids;
    a.evict_ids = mp->evict_ids;
    a.evict_ids_user = evicted_ids;
    a.ln_s_init = mp->ln_s_init;
    a.logit_init = mp->logit_init;
    auto rebuild = [&](long long q0, long long q1, long long r_off, long long e_off) {
        if (q1 <= q0) return;
        StageTimer tm(ctx, ST_MAP_REBUILD, s);
        a.q_begin = q0;
        a.q_end = q1;
        a.reload_off = r_off;
        a.evict_off = e_off;
        hipLaunchKernelGGL(map_rebuild_kernel, dim3(grid_of(q1 - q0), 3 * a.chunks), dim3(kMapThreads), 0, s, a, m);
    };
    // offloaded rows [0, e) of the staging into the host store, on the caller's thread
    auto store_offloads = [&](long long e) -> int {
        if (e > 0) {
            StageTimer tm(ctx, ST_MAP_COPY, s);
            if (hipMemcpyAsync(mp->pinned, mp->stage_out, row_f * sizeof(float) * (size_t)e, hipMemcpyDeviceToHost, s) !=
                    hipSuccess ||
                hipMemcpyAsync(mp->h_evicted, mp->evict_ids, 4 * (size_t)e, hipMemcpyDeviceToHost, s) != hipSuccess)
                return ctx_record_hip(ctx, hipGetLastError());
        }
        if (hipStreamSynchronize(s) != hipSuccess) return ctx_record_hip(ctx, hipGetLastError());
        parallel_rows(e, 2048, [&](long long b, long long f) {
            for (long long r = b; r < f; ++r)
                memcpy(mp->store + (size_t)mp->h_evicted[r] * row_f, mp->pinned + r * row_f, row_f * sizeof(float));
        });
        return AGS_OK;
    };
    if (chunked) {
        // listed rows in chunks of S: each holds at most S reloaded and S offloaded rows
        const long long R0 = n_in + n_new;
        auto clampr = [&](long long x) { return x < 0 ? 0 : (x > n_reload ? n_reload : x); };
        auto evict_before = [&](long long q, long long* e) -> int {  // offloaded rows listed before q
            uint32_t v = 0;
            if (n_evict > 0 && q < l.n_list &&
                (hipMemcpyAsync(&v, mp->evict_pos + q, 4, hipMemcpyDeviceToHost, s) != hipSuccess ||
                 hipStreamSynchronize(s) != hipSuccess))
                return ctx_record_hip(ctx, hipGetLastError());
            *e = n_evict == 0 ? 0 : (q >= l.n_list ? n_evict : (long long)v);
            return AGS_OK;
        };
        for (long long q0 = 0; q0 < l.n_list; q0 += S) {
            const long long q1 = q0 + S < l.n_list ? q0 + S : l.n_list;
            const long long r0 = clampr(q0 - R0), r1 = clampr(q1 - R0);
            long long e0 = 0, e1 = 0;
            int rc = evict_before(q0, &e0);
            if (rc == AGS_OK) rc = evict_before(q1, &e1);
            if (rc == AGS_OK) rc = stage_reloads(r0, r1);
            if (rc != AGS_OK) return rc;
            rebuild(q0, q1, r0, e0);
            rc = store_offloads(e1 - e0);
            if (rc != AGS_OK) return rc;
        }
    } else {
        rebuild(0, l.n_list, 0, 0);
        if (n_evict > 0) {
            // the offloaded rows (device staging, written by the rebuild) go to pinned memory on
            // the copy stream, which waits for the rebuild; the caller's stream goes on at once
            if (hipEventRecord(mp->ev_ready, s) != hipSuccess ||
                hipStreamWaitEvent(mp->cstream, mp->ev_ready, 0) != hipSuccess)
                return ctx_record_hip(ctx, hipGetLastError());
            {
                StageTimer tm(ctx, ST_MAP_COPY, mp->cstream);  // the copies alone, after the wait
                if (hipMemcpyAsync(mp->pinned, mp->stage_out, row_f * sizeof(float) * (size_t)n_evict,
                                   hipMemcpyDeviceToHost, mp->cstream) != hipSuccess ||
                    hipMemcpyAsync(mp->h_evicted, mp->evict_ids, 4 * (size_t)n_evict, hipMemcpyDeviceToHost,
                                   mp->cstream) != hipSuccess ||
                    hipEventRecord(mp->ev_copied, mp->cstream) != hipSuccess)
                    return ctx_record_hip(ctx, hipGetLastError());
            }
            // a host thread waits for the copy and puts the rows into the host store while the
            // caller goes on; the next call (or ags_map_sync / read_store / destroy) joins it first
            auto write_rows = [mp, n_evict, row_f]() {
                if (hipEventSynchronize(mp->ev_copied) != hipSuccess) {
                    mp->flush_err.store(1);
                    return;
                }
                parallel_rows(n_evict, 2048, [&](long long b, long long e) {
                    for (long long r = b; r < e; ++r)
                        memcpy(mp->store + (size_t)mp->h_evicted[r] * row_f, mp->pinned + r * row_f,
                               row_f * sizeof(float));
                });
            };
            try {
                mp->flush = std::thread(write_rows);
            } catch (...) {
                write_rows();  // no thread available: write them now
            }
        }
    }
    // the resident set is complete when the call returns
    if (hipStreamSynchronize(s) != hipSuccess) return ctx_record_hip(ctx, hipGetLastError());
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return ctx_record_hip(ctx, e);
    mp->n_ids += n_new;
    mp->n_resident = n_keep;
    mp->n_offloaded += n_evict - n_reload;
    mp->last_frame = frame;
    counts->n_ids = mp->n_ids;
    counts->n_resident = n_keep;
    counts->n_new = n_new;
    counts->n_reloaded = n_reload;
    counts->n_evicted = n_evict;
    counts->n_offloaded = mp->n_offloaded;
    counts->n_retired = 0;
    return AGS_OK;
}

int ags_map_lifecycle(ags_map* mp, const int32_t* ids, const uint8_t* actions, int64_t n,
                      const ags_gaussians* rows, const ags_gaussians* rows_m, const ags_gaussians* rows_v,
                      ags_gaussians* out, ags_gaussians* out_m, ags_gaussians* out_v, int32_t* out_ids,
                      ags_map_counts* counts, void* stream) {
    if (!mp || !counts) return AGS_ERR_INVALID_ARG;
    if (n != mp->n_resident || (n > 0 && (!ids || !actions || !out_ids))) return AGS_ERR_INVALID_ARG;
    const int deg = mp->cfg.sh_degree;
    if (!map_gaussians_ok(rows, deg) || !map_gaussians_ok(rows_m, deg) || !map_gaussians_ok(rows_v, deg) ||
        !map_gaussians_ok(out, deg) || !map_gaussians_ok(out_m, deg) || !map_gaussians_ok(out_v, deg))
        return AGS_ERR_INVALID_ARG;
    if (rows_m->n != rows->n || rows_v->n != rows->n || out_m->n != out->n || out_v->n != out->n)
        return AGS_ERR_INVALID_ARG;
    ags_ctx* ctx = mp->ctx;
    long long n_new = 0, n_out = 0;
    if (n > 0) {
        if (hipSetDevice(mp->device) != hipSuccess) return ctx_record_hip(ctx, hipGetLastError());
        hipStream_t s = (hipStream_t)stream;
        const MapDev m = dev_of(mp);
        LifeArgs a;
        a.ids = ids;
        a.actions = actions;
        a.n = n;
        a.n_ids = mp->n_ids;
        a.outs = mp->keys[0];
        a.extra = mp->keys[1];
        a.out_pos = mp->vals[0];
        a.new_rank = mp->vals[1];
        a.bad = mp->counters + 2;
        ScanTemp st;
        st.block_sums = mp->block_sums;
        const unsigned g = grid_of(n);
        StageTimer tm(ctx, ST_LIFECYCLE, s);
        launch_fill_u32(mp->counters, 0u, 4, s);
        hipLaunchKernelGGL(map_life_count_kernel, dim3(g), dim3(kMapThreads), 0, s, a, m);
        hipLaunchKernelGGL(map_ids_unmark_kernel, dim3(g), dim3(kMapThreads), 0, s, m, ids, (long long)n,
                           (long long)mp->n_ids);
        launch_scan(a.outs, nullptr, false, a.out_pos, n, nullptr, mp->counters, st, s);
        launch_scan(a.extra, nullptr, false, a.new_rank, n, nullptr, mp->counters + 1, st, s);
        uint32_t hc[4];
        if (hipMemcpyAsync(hc, mp->counters, sizeof(hc), hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            return ctx_record_hip(ctx, hipGetLastError());
        n_out = hc[0];
        n_new = hc[1];
        // nothing changed on a refusal
        if (hc[2] != 0 || rows->n < n_out || out->n < n_out) return AGS_ERR_INVALID_ARG;
        if (mp->n_ids + n_new > mp->cfg.max_ids) return AGS_ERR_CAPACITY;
        hipLaunchKernelGGL(map_life_apply_kernel, dim3(g), dim3(kMapThreads), 0, s, a, m, out_ids);
        hipLaunchKernelGGL(map_life_min_kernel, dim3(grid_of(mp->n_ids + n_new)), dim3(kMapThreads), 0, s, m,
                           (long long)(mp->n_ids + n_new));
        hipLaunchKernelGGL(map_life_settle_kernel, dim3(g), dim3(kMapThreads), 0, s, a, m);
        if (n_out > 0) {
            PackArgs pk;
            const ags_gaussians* ins[3] = {rows, rows_m, rows_v};
            ags_gaussians* outs[3] = {out, out_m, out_v};
            for (int t = 0; t < 3; ++t) {
                const float* src[5] = {ins[t]->means, ins[t]->log_scales, ins[t]->quats, ins[t]->opacity_logits,
                                       ins[t]->sh};
                float* dst[5] = {outs[t]->means, outs[t]->log_scales, outs[t]->quats, outs[t]->opacity_logits,
                                 outs[t]->sh};
                for (int f = 0; f < 5; ++f) {
                    pk.in[t][f] = src[f];
                    pk.out[t][f] = dst[f];
                }
            }
            pk.sn = rows->n;
            pk.dn = n_out;
            pk.k3 = 3 * (deg + 1) * (deg + 1);
            pk.chunks = 1 + (pk.k3 + kMapRows - 1) / kMapRows;
            hipLaunchKernelGGL(map_life_pack_kernel, dim3(grid_of(n_out), 3 * pk.chunks), dim3(kMapThreads), 0, s,
                               pk);
        }
        if (hipStreamSynchronize(s) != hipSuccess) return ctx_record_hip(ctx, hipGetLastError());
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return ctx_record_hip(ctx, e);
    }
    mp->n_ids += n_new;
    mp->n_resident = n_out;
    counts->n_ids = mp->n_ids;
    counts->n_resident = n_out;
    counts->n_new = n_new;
    counts->n_reloaded = 0;
    counts->n_evicted = 0;
    counts->n_offloaded = mp->n_offloaded;
    counts->n_retired = n + n_new - n_out;
    return AGS_OK;
}

int ags_map_export(ags_map* mp, uint64_t* keys, int32_t* last_used, uint8_t* resident, uint64_t* table_keys,
                   int32_t* table_ids, int64_t table_slots, int64_t* n_ids, int64_t* n_slots) {
    if (!mp) return AGS_ERR_INVALID_ARG;
    if ((table_keys || table_ids) && table_slots < mp->slots) return AGS_ERR_INVALID_ARG;
    if (hipSetDevice(mp->device) != hipSuccess) return ctx_record_hip(mp->ctx, hipGetLastError());
    const size_t I = (size_t)mp->n_ids;
    if (hipDeviceSynchronize() != hipSuccess) return ctx_record_hip(mp->ctx, hipGetLastError());
    if ((keys && I && hipMemcpy(keys, mp->id_key, 8 * I, hipMemcpyDeviceToHost) != hipSuccess) ||
        (last_used && I && hipMemcpy(last_used, mp->id_last, 4 * I, hipMemcpyDeviceToHost) != hipSuccess) ||
        (resident && I && hipMemcpy(resident, mp->id_res, I, hipMemcpyDeviceToHost) != hipSuccess) ||
        (table_keys && hipMemcpy(table_keys, mp->tab_keys, 8 * (size_t)mp->slots, hipMemcpyDeviceToHost) !=
                           hipSuccess) ||
        (table_ids &&
         hipMemcpy(table_ids, mp->tab_vals, 4 * (size_t)mp->slots, hipMemcpyDeviceToHost) != hipSuccess))
        return ctx_record_hip(mp->ctx, hipGetLastError());
    if (n_ids) *n_ids = mp->n_ids;
    if (n_slots) *n_slots = mp->slots;
    return AGS_OK;
}

int ags_map_sync(ags_map* mp) {
    if (!mp) return AGS_ERR_INVALID_ARG;
    return flush_join(mp);
}

int ags_map_read_store(ags_map* mp, const int32_t* ids, int64_t n, float* rows) {
    if (!mp || n < 0 || (n > 0 && (!ids || !rows))) return AGS_ERR_INVALID_ARG;
    if (n == 0) return AGS_OK;
    if (flush_join(mp) != AGS_OK) return AGS_ERR_HIP;
    std::vector<uint8_t> res((size_t)mp->n_ids);
    if (hipSetDevice(mp->device) != hipSuccess || hipDeviceSynchronize() != hipSuccess ||
        (mp->n_ids > 0 && hipMemcpy(res.data(), mp->id_res, (size_t)mp->n_ids, hipMemcpyDeviceToHost) != hipSuccess))
        return ctx_record_hip(mp->ctx, hipGetLastError());
    const size_t row_f = (size_t)3 * mp->F;
    for (int64_t k = 0; k < n; ++k)
        if (ids[k] < 0 || ids[k] >= mp->n_ids || res[(size_t)ids[k]]) return AGS_ERR_INVALID_ARG;
    for (int64_t k = 0; k < n; ++k) memcpy(rows + k * row_f, mp->store + (size_t)ids[k] * row_f, row_f * sizeof(float));
    return AGS_OK;
}

}  // extern "C"
