// Tile rasterisation of all views in one launch: forward compositing and its adjoint.
//
// A workgroup owns one T x T tile of one view (the global tile id selects the view), so a
// rig's views and a set of submaps share one launch.  The tile's depth-ordered Gaussian
// list is streamed through LDS in batches; every lane reads the same record (LDS
// broadcast) and composites its pixel(s) front to back (Sec. III-B, standard 3DGS):
//   power = -1/2 (a dx^2 + c dy^2) - b dx dy, (dx, dy) = (u, v) - pixel centre
//   alpha = min(alpha_max, o e^power), skipped when power > 0 or alpha < alpha_min
//   T' = T (1 - alpha); stop (excluding this Gaussian) when T' < t_min
//   C += alpha T rgb; D += alpha T z; T = T'
// and the accumulated alpha A = sum alpha T is written as 1 - T_final (the same sum, not
// accumulated in the loop).
// A workgroup stops fetching batches once every pixel has stopped, and a wave whose lanes
// have all stopped skips the rest of a batch.  The forward keeps 8 bytes per pixel
// (final T and the list position of the last contributor) so the backward recomputes
// transmittance instead of storing per-pixel blend lists.
//
// The backward walks the list back to front from the last contributor, recovering
// T_k = T_{k+1} / (1 - alpha_k) and accumulating suffix sums S = sum_{j>k} w_j f_j:
//   dL/dalpha_k = T_k (gC . c_k + gD z_k + gA)
//                 - (gC . S^C + gD S^D + gA S^A + T_final gC . bg) / (1 - alpha_k)
// (the bracket is kept as one running sum U), then chains through alpha = o e^power (unless
// clamped) to the opacity, h = dL/do = e^power dL/dalpha, and to dL/dpower = o h, of which
// it keeps five pixel moments without the factor o (sum h dx, h dy, h dx^2, h dx dy,
// h dy^2); the projection backward applies o and turns them into the centre and conic
// adjoints.  dL/drgb_k = w_k gC, dL/dz_k = w_k gD.  The ten per-Gaussian
// sums of a wave are reduced with a transposing butterfly to ten lanes.  With LDS batches of
// at most 64 records those lanes add them into the batch's LDS accumulator of that Gaussian
// (the workgroup's waves merge there), and after the batch one global atomic per (Gaussian,
// non-zero sum) adds the workgroup's total into the pair's 64-byte adjoint row, so each row
// is updated once per tile; with larger batches (where the accumulator's LDS would cut the
// number of resident workgroups) one atomic instruction of the ten lanes per wave updates
// the row.
#include "common.h"

namespace ags {

struct TileCoord {
    int b, px0, py0, W, H;
    long long pix0;  // first pixel of the view in the flat image buffers
};

__device__ __forceinline__ TileCoord tile_coord(const ViewTable& vt, int tile) {
    TileCoord c;
    c.b = view_of_tile(vt, tile);
    int local = tile - vt.tile_base[c.b];
    int ntx = vt.ntx[c.b];
    c.px0 = (local % ntx) * vt.tile;
    c.py0 = (local / ntx) * vt.tile;
    c.W = vt.width[c.b];
    c.H = vt.height[c.b];
    c.pix0 = vt.pix_base[c.b];
    return c;
}

// Each wave owns a rectangular block of the tile: 8 columns x 8 PPT rows when the tile has
// enough waves for its 8-wide column strips, else the full tile width.  Lane l covers
// column l % BW and PPT vertically adjacent rows.  The per-record wave mask below lets a
// whole wave skip Gaussians whose footprint box misses its block.
template <int T, int PPT>
struct WaveGrid {
    static constexpr int NT = T * T / PPT;
    static constexpr int NW = NT / 64;
    static constexpr int BW = (NW >= T / 8) ? 8 : T;
    static constexpr int COLS = T / BW;
    static constexpr int BH = 64 * PPT / BW;
    static_assert(COLS * (T / BH) == NW, "wave blocks must tile the tile");
};

// BLOCKS = false: row strips (thread t covers column t % T and PPT rows), used by the
// forward, where full-width rows keep the output writes coalesced.  BLOCKS = true: the wave
// blocks above, used by the backward together with the wave mask.
template <int T, int PPT, bool BLOCKS>
__device__ __forceinline__ void pixel_of(int t, int k, int& x, int& y) {
    if (BLOCKS) {
        using G = WaveGrid<T, PPT>;
        const int w = t >> 6, l = t & 63;
        x = (w % G::COLS) * G::BW + l % G::BW;
        y = (w / G::COLS) * G::BH + (l / G::BW) * PPT + k;
    } else {
        x = t % T;
        y = (t / T) * PPT + k;
    }
}

// Bit w set when the record's pixel footprint box (the binning rectangle, clamped to the
// image) intersects the pixels of wave w in the tile at (px0, py0): its block (BLOCKS) or
// its rows (row strips).  (The forward does not use it: testing it per entry cost more
// than the skipped entries saved there.)
template <int T, int PPT, bool BLOCKS>
__device__ __forceinline__ uint32_t wave_mask(float u, float v, float ex, float ey, int W, int H, int px0,
                                              int py0) {
    using G = WaveGrid<T, PPT>;
    const float fx0 = floorf(__fsub_rn(__fsub_rn(u, ex), 0.5f));
    const float fx1 = ceilf(__fsub_rn(__fadd_rn(u, ex), 0.5f));
    const float fy0 = floorf(__fsub_rn(__fsub_rn(v, ey), 0.5f));
    const float fy1 = ceilf(__fsub_rn(__fadd_rn(v, ey), 0.5f));
    // relative to the tile, clamped to [-1, T]
    const int x0 = (int)fminf(fmaxf(fx0 - (float)px0, -1.f), (float)T);
    const int x1 = (int)fminf(fmaxf(fx1 - (float)px0, -1.f), (float)T);
    const int y0 = (int)fminf(fmaxf(fy0 - (float)py0, -1.f), (float)T);
    const int y1 = (int)fminf(fmaxf(fy1 - (float)py0, -1.f), (float)T);
    uint32_t m = 0;
    if (BLOCKS) {
#pragma unroll
        for (int w = 0; w < G::NW; ++w) {
            const int bx0 = (w % G::COLS) * G::BW, by0 = (w / G::COLS) * G::BH;
            if (x0 <= bx0 + G::BW - 1 && x1 >= bx0 && y0 <= by0 + G::BH - 1 && y1 >= by0) m |= 1u << w;
        }
    } else {
        constexpr int RW = 64 * PPT / T;  // rows per wave (>= T: one wave holds the tile)
        if (x0 <= T - 1 && x1 >= 0) {
#pragma unroll
            for (int w = 0; w < G::NW; ++w)
                if (y0 <= w * RW + RW - 1 && y1 >= w * RW) m |= 1u << w;
        }
    }
    (void)W;
    (void)H;
    return m;
}

// Copy record q into LDS in the form the per-pixel loops use: the conic (a, b, c) becomes
// log2(e) (-a/2, -b, -c/2), so the exponent in base 2, p2 = dx (A' dx + B' dy) + C' dy^2,
// costs five operations and e^power = exp2(p2) is one instruction; the footprint extent is
// replaced by the exponent floor log2(alpha_min / o) - kPreTestMargin and by the mask of wave
// blocks its footprint box touches.  Both kernels keep a (pixel, Gaussian) pair exactly when
// p2 <= 0 and alpha = min(alpha_max, o exp2(p2)) >= alpha_min, in float32, so their decisions
// agree; the backward tests the exponent floor first to skip whole entries.  A kept pair has
// o exp2(p2) >= alpha_min, so p2 >= log2(alpha_min / o) less the float32 rounding of the
// product and of exp2 (a few 1e-7), and the computed floor is within ~1e-6 of the exact
// log2: the 1e-4 margin keeps every kept pair above the floor, so the pre-test never
// changes a decision; every skipped pair has alpha < alpha_min.
// LDS layout (64 B, read at non-negative offsets from one per-lane address):
//   [0] = (wave mask bits, r, g, b) in the backward, (z, r, g, b) in the forward,
//   [1] = (u, v, -a/2 log2e, -b log2e), [2] = (-c/2 log2e, o, z, exponent floor),
//   [3] = (pair id, z^2, address of the pair's 2D adjoint row (backward)).
// The forward reads 24 bytes of an entry ([1] and the first half of [2]) before its keep
// test and [0] only for a pixel that takes the Gaussian.
struct alignas(16) SRec {
    float4 m, g0, g1;
    uint32_t q;
    float z2;
    float* row;  // the pair's 2D adjoint row (backward)
};

constexpr float kPreTestMargin = 1e-4f;
template <int T, int PPT, bool BLOCKS>
__device__ __forceinline__ uint32_t stage_record(const float* records, uint32_t q, float amin, int W, int H,
                                                 int px0, int py0, SRec& dst, float* grad2d = nullptr) {
    const float4* r = reinterpret_cast<const float4*>(records + (long long)q * kRecFloats);
    const float4 r0 = r[0], r1 = r[1], r2 = r[2];
    constexpr float kLog2e = 1.4426950408889634f;
    const uint32_t m = BLOCKS ? wave_mask<T, PPT, BLOCKS>(r0.x, r0.y, r1.w, r2.x, W, H, px0, py0) : ~0u;
    dst.m = make_float4(BLOCKS ? __uint_as_float(m) : r1.z, r2.y, r2.z, r2.w);
    dst.g0 = make_float4(r0.x, r0.y, -0.5f * kLog2e * r0.z, -kLog2e * r0.w);
    dst.g1 = make_float4(-0.5f * kLog2e * r1.x, r1.y, r1.z, __log2f(amin / r1.y) - kPreTestMargin);
    dst.q = q;
    dst.z2 = r1.z * r1.z;
    if (BLOCKS) dst.row = grad2d + (long long)q * kGrad2dStride;
    return m;
}

// Makes the record's fields live at this point, so all of its LDS reads are issued together
// (one round trip) instead of being deferred past the wave-uniform tests that use them.
__device__ __forceinline__ void use_record(const float4& a, const float4& b) {
    asm volatile("" ::"v"(a.x), "v"(a.y), "v"(a.z), "v"(a.w), "v"(b.x), "v"(b.y), "v"(b.z), "v"(b.w));
}
__device__ __forceinline__ void use_record(const float4& a, const float4& b, const float4& c) {
    use_record(a, b);
    asm volatile("" ::"v"(c.x), "v"(c.y), "v"(c.z), "v"(c.w));
}

// Keeps a value in a vector register from here on, so an LDS address derived from it is
// advanced with one vector add per iteration instead of being rebuilt from scalars.
template <typename V>
__device__ __forceinline__ void in_vgpr(V& v) {
    asm volatile("" : "+v"(v));
}

__device__ __forceinline__ float power_of(const float4& r0, const float4& r1, float dx, float dy) {
    return dx * (r0.z * dx + r0.w * dy) + r1.x * dy * dy;
}

// S2: also output the rendered depth variance sum w z^2 - (sum w z)^2 (rendered-variance
// LiDAR term), accumulated without cancellation: the weighted scatter S about the running
// normalised mean m (A' = A + w, m' = m + (z - m) w / A', S' = S + w (z - m)(z - m')), then
// sum w z^2 - (A m)^2 = S + A (1 - A) m^2 with 1 - A = the final transmittance.
template <int T, int PPT, int M, bool S2>
__global__ __launch_bounds__(T* T / PPT) void raster_fwd_kernel(RasterArgs a) {
    constexpr int NT = T * T / PPT;
    __shared__ SRec srec[M];
    const uint32_t wt = a.work[blockIdx.x];
    if (wt == kNoTile) return;  // padding of a shorter XCD list (whole workgroup)
    const int tile = (int)wt;
    const TileCoord tc = tile_coord(a.vt, tile);
    const uint32_t start = __builtin_amdgcn_readfirstlane(a.ranges[2 * tile]);
    const uint32_t end = __builtin_amdgcn_readfirstlane(a.ranges[2 * tile + 1]);
    const int tid = threadIdx.x;

    // A pixel that has stopped (or lies outside the image) gets cx = +inf: its exponent is
    // then -inf (or NaN), below every threshold, so it keeps no further Gaussian without a
    // separate flag test.
    constexpr float kStopped = __builtin_huge_valf();
    float cx[PPT], cy[PPT], Tr[PPT], C0[PPT], C1[PPT], C2[PPT], D[PPT], A[PPT], Mn[PPT], Sc[PPT];
    uint32_t last[PPT];
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
        int lx, ly;
        pixel_of<T, PPT, false>(tid, k, lx, ly);
        const int px = tc.px0 + lx, py = tc.py0 + ly;
        cx[k] = (px < tc.W && py < tc.H) ? (float)px + 0.5f : kStopped;
        cy[k] = (float)py + 0.5f;
        Tr[k] = 1.f;
        C0[k] = C1[k] = C2[k] = D[k] = A[k] = Mn[k] = Sc[k] = 0.f;
        last[k] = 0;
    }
    const float amin = a.st.alpha_min, tmin = a.st.t_min;
    const float amax = __builtin_canonicalizef(a.st.alpha_max);

    for (uint32_t bs = start; bs < end; bs += M) {
        bool any = false;
#pragma unroll
        for (int k = 0; k < PPT; ++k) any |= cx[k] != kStopped;
        if (__syncthreads_count(any) == 0) break;
#pragma unroll
        for (int l = tid; l < M; l += NT) {
            const uint32_t e = bs + l;
            if (e < end)
                stage_record<T, PPT, false>(a.records, a.tile_pairs[e], amin, tc.W, tc.H, tc.px0, tc.py0,
                                            srec[l]);
        }
        __syncthreads();
        const uint32_t bend = end - bs > (uint32_t)M ? bs + M : end;
        const char* sbase = reinterpret_cast<const char*>(srec);
        uint32_t off = 0;  // byte offset of record e - bs in LDS
        in_vgpr(off);
        // entries in groups of eight: the later records are read at immediate offsets from the
        // first's LDS address, so the address advances once per group, and the wave's early
        // exit is tested once per group (entries past a wave's stop keep nothing: a stopped
        // pixel's exponent is -inf or NaN)
        auto entry = [&](const SRec& r, uint32_t e) {
            const float4 r0 = r.g0;
            const float2 r1 = *reinterpret_cast<const float2*>(&r.g1);  // (C', o)
            use_record(r0, make_float4(r1.x, r1.y, 0.f, 0.f));
#pragma unroll
            for (int k = 0; k < PPT; ++k) {
                // one predicate, one branch: the exp is cheap next to divergent control
                const float dx = r0.x - cx[k], dy = r0.y - cy[k];
                const float p2 = dx * (r0.z * dx + r0.w * dy) + r1.x * dy * dy;
                const float alpha = fminf(amax, r1.y * __builtin_amdgcn_exp2f(p2));
                const bool keep = p2 <= 0.f && alpha >= amin;
                if (keep) {
                    // stop (once per pixel) before a Gaussian that would take T below t_min;
                    // the tested T (1 - alpha), one rounding, is the next T
                    const float Tn = __builtin_fmaf(-alpha, Tr[k], Tr[k]);
                    const bool go = Tn >= tmin;
                    cx[k] = go ? cx[k] : kStopped;  // +inf marks the pixel stopped
                    in_vgpr(cx[k]);                 // one select here, not moves in both branches
                    if (go) {
                        const float4 rc = r.m;  // (z, r, g, b)
                        const float w = alpha * Tr[k];
                        C0[k] += w * rc.y;
                        C1[k] += w * rc.z;
                        C2[k] += w * rc.w;
                        D[k] += w * rc.x;
                        if (S2) {
                            A[k] += w;
                            const float dz = rc.x - Mn[k];
                            Mn[k] += dz * (w * __builtin_amdgcn_rcpf(A[k]));
                            Sc[k] += w * dz * (rc.x - Mn[k]);
                        }
                        Tr[k] = Tn;
                        last[k] = e - start + 1;
                    }
                }
            }
        };
        auto wave_live = [&]() {
            bool live = false;
#pragma unroll
            for (int k = 0; k < PPT; ++k) live |= cx[k] != kStopped;
            return __ballot(live) != 0ull;  // wave-uniform: false once every pixel has stopped
        };
        for (uint32_t e = bs; e < bend; e += 8, off += 8 * sizeof(SRec)) {
            if (!wave_live()) break;
            entry(*reinterpret_cast<const SRec*>(sbase + off), e);
#pragma unroll
            for (int g = 1; g < 8; ++g) {
                if (e + g == bend) break;
                entry(*reinterpret_cast<const SRec*>(sbase + off + g * sizeof(SRec)), e + g);
            }
        }
        __syncthreads();
    }
    const long long plane = (long long)tc.W * tc.H;
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
        int lx, ly;
        pixel_of<T, PPT, false>(tid, k, lx, ly);
        if (tc.px0 + lx >= tc.W || tc.py0 + ly >= tc.H) continue;
        const long long p = (long long)(tc.py0 + ly) * tc.W + (tc.px0 + lx);
        const long long gp = tc.pix0 + p;
        float* rgb = a.rgb + 3 * tc.pix0;
        rgb[p] = C0[k] + Tr[k] * a.st.bg0;
        rgb[plane + p] = C1[k] + Tr[k] * a.st.bg1;
        rgb[2 * plane + p] = C2[k] + Tr[k] * a.st.bg2;
        a.depth[gp] = D[k];
        if (S2) a.depth_var[gp] = Sc[k] + A[k] * Tr[k] * Mn[k] * Mn[k];
        a.alpha[gp] = 1.f - Tr[k];
        a.t_final[gp] = Tr[k];
        a.last[gp] = last[k];
        if (a.zero_px[0]) a.zero_px[0][gp] = 0.f;
        if (a.zero_px[1]) a.zero_px[1][gp] = 0.f;
    }
}

// GA: the upstream adjoint has an alpha term (dL/dA); the fused loss never has one.
// S2: the loss has an adjoint for the second depth moment sum w z^2 (rendered variance).
template <int T, int PPT, int M, bool GA, bool S2>
__global__ __launch_bounds__(T* T / PPT) void raster_bwd_kernel(RasterBwdArgs a) {
    constexpr int NT = T * T / PPT;
    // merge the waves' sums in LDS where that keeps the workgroup within 8 KB of LDS
    constexpr bool MERGE = M <= 64 && NT > 64;
    __shared__ SRec srec[M];
    __shared__ float sacc[MERGE ? M * kGrad2d : 1];  // per LDS slot: the workgroup's ten sums
    __shared__ uint32_t sq[2][MERGE ? M : 1];        // the pairs of this batch and the previous
    __shared__ uint32_t smax;
    __shared__ float sred[NT / 64];
    // per wave, one bit per LDS slot of the batch: the record's footprint box meets the wave's
    // block (read into scalar registers once per batch, so an entry's skip test costs no
    // vector instruction and waits on no LDS read)
    constexpr int kWords = (M + 63) / 64;
    __shared__ unsigned long long smask[NT / 64][kWords];
    const uint32_t wt = a.work[blockIdx.x];
    if (wt == kNoTile) return;  // padding of a shorter XCD list (whole workgroup)
    const int tile = (int)wt;
    const TileCoord tc = tile_coord(a.vt, tile);
    const uint32_t start = __builtin_amdgcn_readfirstlane(a.ranges[2 * tile]);
    const int tid = threadIdx.x;
    const int lane = __lane_id();
    const int wave = tid >> 6;
    const float amin = a.st.alpha_min;

    // U = T_final gC.bg + sum over later contributors j of w_j (gC.c_j + gD z_j + gA)
    float cx[PPT], cy[PPT], Tr[PPT], gC0[PPT], gC1[PPT], gC2[PPT], gD[PPT], gA[PPT], gM[PPT], U[PPT];
    uint32_t last[PPT];
    float loss_part = 0.f;
    uint32_t mylast = 0;
    const long long plane = (long long)tc.W * tc.H;
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
        int lx, ly;
        pixel_of<T, PPT, true>(tid, k, lx, ly);
        const int px = tc.px0 + lx, py = tc.py0 + ly;
        cx[k] = (float)px + 0.5f;
        cy[k] = (float)py + 0.5f;
        gC0[k] = gC1[k] = gC2[k] = gD[k] = gA[k] = gM[k] = 0.f;
        Tr[k] = 1.f;
        last[k] = 0;
        U[k] = 0.f;
        if (px < tc.W && py < tc.H) {
            const long long p = (long long)py * tc.W + px;
            const long long gp = tc.pix0 + p;
            Tr[k] = a.t_final[gp];
            last[k] = a.last[gp];
            if (a.loss_mode) {
                const bool on = a.mask ? (a.mask[gp] != 0) : true;
                if (on) {
                    const float sc = a.l1_scale[tc.b];
                    const float* rgb = a.rgb + 3 * tc.pix0;
                    const float* gt = a.gt_rgb + 3 * tc.pix0;
                    const float d0 = rgb[p] - gt[p];
                    const float d1 = rgb[plane + p] - gt[plane + p];
                    const float d2 = rgb[2 * plane + p] - gt[2 * plane + p];
                    gC0[k] = d0 > 0.f ? sc : (d0 < 0.f ? -sc : 0.f);
                    gC1[k] = d1 > 0.f ? sc : (d1 < 0.f ? -sc : 0.f);
                    gC2[k] = d2 > 0.f ? sc : (d2 < 0.f ? -sc : 0.f);
                    loss_part += sc * (fabsf(d0) + fabsf(d1) + fabsf(d2));
                }
                if (a.d_rgb) {  // D-SSIM adjoint (already zero outside the mask)
                    const float* g = a.d_rgb + 3 * tc.pix0;
                    gC0[k] += g[p];
                    gC1[k] += g[plane + p];
                    gC2[k] += g[2 * plane + p];
                }
                if (a.d_depth) gD[k] = a.d_depth[gp];
                if (S2) gM[k] = a.d_depth2[gp];
            } else {
                if (a.d_rgb) {
                    const float* g = a.d_rgb + 3 * tc.pix0;
                    gC0[k] = g[p];
                    gC1[k] = g[plane + p];
                    gC2[k] = g[2 * plane + p];
                }
                if (a.d_depth) gD[k] = a.d_depth[gp];
                if (GA) gA[k] = a.d_alpha[gp];
            }
            U[k] = Tr[k] * (gC0[k] * a.st.bg0 + gC1[k] * a.st.bg1 + gC2[k] * a.st.bg2);
            mylast = max(mylast, last[k]);
        }
    }
    if (a.loss_mode) {
        // block sum of the L1 partials (deterministic order)
        float s = wave_sum(loss_part);
        if (lane == 0) sred[tid >> 6] = s;
    }
    if (tid == 0) smax = 0;
    if (MERGE)
        for (int l = tid; l < M * kGrad2d; l += NT) sacc[l] = 0.f;
    __syncthreads();
    atomicMax(&smax, mylast);
    if (a.loss_mode && tid == 0) {
        float s = 0.f;
        for (int w = 0; w < NT / 64; ++w) s += sred[w];
        a.loss_partials[tile] = s;
    }
    __syncthreads();
    const uint32_t maxlast = smax;
    // wave-uniform bound: entries at or past every lane's last contributor are skipped
    uint32_t wlast = mylast;
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) wlast = max(wlast, (uint32_t)__shfl_xor((int)wlast, o, 64));
    const int wl = (int)__builtin_amdgcn_readfirstlane(wlast);

    const float amax = __builtin_canonicalizef(a.st.alpha_max);
    // lane L ends the reduction holding slot (L >> 2) & 15; value v of the ten sums sits in
    // slot kSlot[v % 5] + 8 (v / 5), see wave_transpose_sum10
    const int slot = (lane >> 2) & 15, sl = slot & 7;
    const bool red_lane = (lane & 3) == 0 && sl != 3 && sl < 6;
    const int red_val = (sl < 3 ? sl : sl - 1) + 5 * (slot >> 3);

    // the batch's totals into the pairs' rows, one global atomic per (Gaussian, non-zero sum);
    // the accumulator is left zero for the next batch
    auto flush = [&](int n, const uint32_t* q) {
        for (int l = tid; l < n * kGrad2d; l += NT) {
            const float x = sacc[l];
            if (x != 0.f) {
                const int e = l / kGrad2d;
                atomicAdd(a.grad2d + (long long)q[e] * kGrad2dStride + (l - e * kGrad2d), x);
                sacc[l] = 0.f;
            }
        }
    };
    int prev_n = 0, buf = 0;
    for (int hi = (int)maxlast; hi > 0; hi -= M, buf ^= 1) {
        const int lo = hi - M > 0 ? hi - M : 0;
        if (MERGE) flush(prev_n, sq[buf ^ 1]);  // the previous batch, while this one is staged
        for (int base = 0; base < hi - lo; base += NT) {  // workgroup-uniform trip count
            const int l = base + tid;
            uint32_t m = 0;
            if (l < hi - lo) {
                const uint32_t q = a.tile_pairs[start + lo + l];
                m = stage_record<T, PPT, true>(a.records, q, amin, tc.W, tc.H, tc.px0, tc.py0, srec[l], a.grad2d);
                if (MERGE) sq[buf][l] = q;
            }
            const int l0 = base + 64 * wave;  // this wave's first slot
            if (l0 < M) {
#pragma unroll
                for (int w = 0; w < NT / 64; ++w) {
                    const unsigned long long bits = __ballot((m >> w) & 1u);
                    if (lane == 0) smask[w][l0 >> 6] = bits;
                }
            }
        }
        prev_n = hi - lo;
        __syncthreads();
        unsigned long long mw[kWords];
#pragma unroll
        for (int x = 0; x < kWords; ++x) {
            const unsigned long long v = smask[wave][x];
            mw[x] = ((unsigned long long)__builtin_amdgcn_readfirstlane((uint32_t)(v >> 32)) << 32) |
                    (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)v);
        }
        const int jtop = min(hi, wl);  // wave-uniform
        // entries in groups of four, back to front: the group's records are read at immediate
        // offsets from the LDS address of its lowest entry, which moves once per group
        auto entry = [&](const SRec& r, int j, int e) {
            if (!((mw[e >> 6] >> (e & 63)) & 1ull)) return;  // wave-uniform
            const float4 rm = r.m, r0 = r.g0, r1 = r.g1;
            float* const row = MERGE ? nullptr : r.row;
            use_record(rm, r0, r1);
            const float z2 = S2 ? r.z2 : 0.f;
            // wave-level pre-test on the exponent alone; the adjoint runs only if some lane
            // passes (every lane that keeps this Gaussian passes: the floor sits a margin below
            // the exact threshold; keeps are decided on alpha below, as in the forward)
            float p2v[PPT];
            bool pass[PPT];
            bool anyp = false;
#pragma unroll
            for (int k = 0; k < PPT; ++k) {
                p2v[k] = power_of(r0, r1, r0.x - cx[k], r0.y - cy[k]);
                pass[k] = (uint32_t)j < last[k] && p2v[k] <= 0.f && p2v[k] >= r1.w;
                anyp |= pass[k];
            }
            if (__ballot(anyp) == 0ull) return;  // wave-uniform
            float g[10];
#pragma unroll
            for (int k = 0; k < PPT; ++k) {
                const float dx = r0.x - cx[k], dy = r0.y - cy[k];
                const float p2 = p2v[k];
                const float G = __builtin_amdgcn_exp2f(p2);  // e^power
                const float araw = r1.y * G;
                const float alpha = fminf(amax, araw);
                const bool keep = pass[k] && alpha >= amin;
                // branch-free: a lane that does not keep this Gaussian runs the same steps
                // with alpha = 0, so its w is 0 and its T and U stay as they are (and every
                // quantity stays finite: alpha <= alpha_max < 1)
                const float ak = keep ? alpha : 0.f;
                const float rom = __builtin_amdgcn_rcpf(1.f - ak);
                const float Tk = Tr[k] * rom;
                const float w = ak * Tk;
                float qv = gC0[k] * rm.y + gC1[k] * rm.z + gC2[k] * rm.w + gD[k] * r1.z;
                if (GA) qv += gA[k];
                if (S2) qv += gM[k] * z2;
                const float ga = Tk * qv - U[k] * rom;  // dL/dalpha
                U[k] += w * qv;
                Tr[k] = Tk;
                // through alpha = o e^power (no gradient where the alpha_max clamp is active):
                // h = dL/do, and dL/dpower = h o, whose factor o the projection backward
                // applies to the five pixel moments kept here (sum h dx, h dy, h dx^2, h dx dy,
                // h dy^2); it turns them into the centre and conic adjoints
                const float h = (keep && araw <= amax) ? ga * G : 0.f;
                const float t1 = h * dx, t2 = h * dy;
                // depth adjoint: d(w z)/dz = w, d(w z^2)/dz = 2 w z
                const float gz = S2 ? gD[k] + 2.f * r1.z * gM[k] : gD[k];
                const float c[10] = {t1, t2, t1 * dx, t1 * dy, t2 * dy, h,
                                     w * gC0[k], w * gC1[k], w * gC2[k], w * gz};
#pragma unroll
                for (int s = 0; s < 10; ++s) g[s] = k == 0 ? c[s] : g[s] + c[s];
            }
            const float tot = wave_transpose_sum10(g);
            if (MERGE) {
                if (red_lane) atomicAdd(&sacc[e * kGrad2d + red_val], tot);
            } else {
                if (red_lane) atomicAdd(row + red_val, tot);
            }
        };
        const char* sbase = reinterpret_cast<const char*>(srec);
        int j = jtop - 1;
        int ofs = (j - 3 - lo) * (int)sizeof(SRec);  // byte offset of the group's lowest entry
        in_vgpr(ofs);
        for (; j >= lo + 3; j -= 4, ofs -= 4 * (int)sizeof(SRec)) {
#pragma unroll
            for (int g = 0; g < 4; ++g)
                entry(*reinterpret_cast<const SRec*>(sbase + ofs + (3 - g) * (int)sizeof(SRec)), j - g, j - g - lo);
        }
        for (; j >= lo; --j) entry(srec[j - lo], j, j - lo);
        __syncthreads();
    }
    if (MERGE) flush(prev_n, sq[buf ^ 1]);
}

// The backward's clears in one launch, when the forward's own zeroing of these accumulators
// cannot be relied on (a second backward of one forward).  Thread g zeroes the adjoint rows of
// the pairs 4 g .. 4 g + 3 that some tile lists (the only rows the raster backward adds to
// and the projection backward reads): one 16-byte load of their counts, then the 64-byte row
// stores of the visible ones, so no store waits on more than one load; then, striding over
// the grid, the dense float buffers (the LiDAR depth and second-moment adjoints).
static_assert(kGrad2dStride == 16, "four float4 stores per row");

__global__ __launch_bounds__(256) void bwd_clear_kernel(BwdClearArgs a) {
    const long long g = (long long)blockIdx.x * 256 + threadIdx.x;
    const long long q0 = 4 * g;
    if (q0 < a.n_pairs) {
        uint32_t c[4];
        if (q0 + 4 <= a.n_pairs) {
            const uint4 v = reinterpret_cast<const uint4*>(a.pair_count)[g];  // 16-byte aligned
            c[0] = v.x; c[1] = v.y; c[2] = v.z; c[3] = v.w;
        } else {
#pragma unroll
            for (int j = 0; j < 4; ++j) c[j] = q0 + j < a.n_pairs ? a.pair_count[q0 + j] : 0u;
        }
        const float4 z = make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            if (!c[j]) continue;
            float4* row = reinterpret_cast<float4*>(a.grad2d + (q0 + j) * kGrad2dStride);
#pragma unroll
            for (int k = 0; k < kGrad2dStride / 4; ++k) row[k] = z;
        }
    }
    const long long stride = (long long)gridDim.x * 256;
    for (int r = 0; r < kBwdClearRegions; ++r)
        for (long long i = g; i < a.zero_n[r]; i += stride) a.zero[r][i] = 0.f;
}

void launch_bwd_clear(const BwdClearArgs& a, hipStream_t s) {
    long long most = (a.n_pairs + 3) / 4;
    for (int r = 0; r < kBwdClearRegions; ++r) {
        const long long t = (a.zero_n[r] + 3) / 4;  // about four floats per thread
        most = t > most ? t : most;
    }
    if (most <= 0) return;
    const long long grid = (most + 255) / 256;
    hipLaunchKernelGGL(bwd_clear_kernel, dim3((unsigned)grid), dim3(256), 0, s, a);
}

int raster_blocks(const ViewTable& vt) {
    const int n = vt.tile_base[vt.n_views];
    if (n <= 0) return 0;
    const int strips = (n + kWorkStrip - 1) / kWorkStrip;
    return 8 * ((strips + 7) / 8) * kWorkStrip;  // 8 XCD lists of equal (maximum) length
}

#define AGS_RASTER_CONFIGS(X) \
    X(8, 1, 64)               \
    X(8, 1, 128)              \
    X(16, 1, 128)             \
    X(16, 1, 256)             \
    X(16, 2, 64)              \
    X(16, 2, 128)             \
    X(16, 2, 256)             \
    X(16, 4, 64)              \
    X(32, 4, 256)             \
    X(32, 2, 512)

int raster_shapes(int* tile, int* ppt, int* batch, int n_max) {
    int n = 0;
#define X(t_, p_, m_)             \
    if (n < n_max) {              \
        tile[n] = t_;             \
        ppt[n] = p_;              \
        batch[n] = m_;            \
    }                             \
    ++n;
    AGS_RASTER_CONFIGS(X)
#undef X
    return n;
}

int launch_raster_fwd(const RasterArgs& a, int T, int batch, int ppt, hipStream_t s) {
    const int nb = raster_blocks(a.vt);
    if (nb <= 0) return 0;
#define X(t_, p_, m_)                                                                              \
    if (T == t_ && ppt == p_ && batch == m_) {                                                     \
        if (a.depth_var)                                                                           \
            hipLaunchKernelGGL((raster_fwd_kernel<t_, p_, m_, true>), dim3(nb), dim3(t_ * t_ / p_), 0, s, a); \
        else                                                                                       \
            hipLaunchKernelGGL((raster_fwd_kernel<t_, p_, m_, false>), dim3(nb), dim3(t_ * t_ / p_), 0, s, a); \
        return 0;                                                                                  \
    }
    AGS_RASTER_CONFIGS(X)
#undef X
    return AGS_ERR_NOT_SUPPORTED;
}

int launch_raster_bwd(const RasterBwdArgs& a, int T, int batch, int ppt, hipStream_t s) {
    const int nb = raster_blocks(a.vt);
    if (nb <= 0) return 0;
    const bool ga = !a.loss_mode && a.d_alpha != nullptr;
    const bool m2 = a.loss_mode && a.d_depth2 != nullptr;
#define X(t_, p_, m_)                                                                                      \
    if (T == t_ && ppt == p_ && batch == m_) {                                                             \
        if (ga)                                                                                            \
            hipLaunchKernelGGL((raster_bwd_kernel<t_, p_, m_, true, false>), dim3(nb), dim3(t_ * t_ / p_), 0, s, a); \
        else if (m2)                                                                                       \
            hipLaunchKernelGGL((raster_bwd_kernel<t_, p_, m_, false, true>), dim3(nb), dim3(t_ * t_ / p_), 0, s, a); \
        else                                                                                               \
            hipLaunchKernelGGL((raster_bwd_kernel<t_, p_, m_, false, false>), dim3(nb), dim3(t_ * t_ / p_), 0, s, a); \
        return 0;                                                                                          \
    }
    AGS_RASTER_CONFIGS(X)
#undef X
    return AGS_ERR_NOT_SUPPORTED;
}

}  // namespace ags
