// Internal declarations shared by the HIP translation units of libagsplat.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/agsplat.h"

namespace ags {

constexpr int kMaxViews = AGS_MAX_VIEWS;
constexpr int kRecFloats = 12;       // projected record: u v a b c o z ex ey r g b
// per-pair 2D adjoint: 5 pixel moments of dL/dpower (turned into the centre and conic
// adjoints by the projection backward), then o, r, g, b, z
constexpr int kGrad2d = 10;
constexpr int kGrad2dStride = 16;  // 64-byte rows: a row is one cache line

// Static per-batch table passed by value to kernels (kernel arguments).
struct ViewTable {
    int n_views;
    int tile;
    int ntx[kMaxViews];
    int nty[kMaxViews];
    int width[kMaxViews];
    int height[kMaxViews];
    int g_begin[kMaxViews];
    int g_end[kMaxViews];
    int tile_base[kMaxViews + 1];
    long long pix_base[kMaxViews + 1];
    long long pair_base[kMaxViews + 1];
};

struct Settings {
    float alpha_min, alpha_max, t_min, blur, z_near, fov_clamp;
    float bg0, bg1, bg2;
};

// Counters at the head of the saved buffer.
enum { CNT_K = 0, CNT_V = 1, CNT_OVERFLOW = 2, CNT_KEFF = 3, CNT_LIVE = 4 };

__device__ __forceinline__ int view_of_pair(const ViewTable& vt, long long q) {
    int b = 0;
    for (int k = 1; k < vt.n_views; ++k)
        if (q >= vt.pair_base[k]) b = k;
    return b;
}

__device__ __forceinline__ int view_of_tile(const ViewTable& vt, int t) {
    int b = 0;
    for (int k = 1; k < vt.n_views; ++k)
        if (t >= vt.tile_base[k]) b = k;
    return b;
}

// Footprint rectangle in tiles of a projected Gaussian (centre u, v; bounding
// half-extents ex, ey), in float32 exactly as written: pixels
// [floor((u - ex) - 0.5), ceil((u + ex) - 0.5)] clamped to the image, then // T.
// Returns false when the rectangle is empty.
__device__ __forceinline__ bool tile_rect(float u, float v, float ex, float ey, int W, int H,
                                          int T, int& tx0, int& ty0, int& tx1, int& ty1) {
    float fx0 = floorf(__fsub_rn(__fsub_rn(u, ex), 0.5f));
    float fx1 = ceilf(__fsub_rn(__fadd_rn(u, ex), 0.5f));
    float fy0 = floorf(__fsub_rn(__fsub_rn(v, ey), 0.5f));
    float fy1 = ceilf(__fsub_rn(__fadd_rn(v, ey), 0.5f));
    int x0 = fx0 < 0.f ? 0 : (fx0 > (float)W ? W : (int)fx0);
    int x1 = fx1 > (float)(W - 1) ? W - 1 : (fx1 < -1.f ? -1 : (int)fx1);
    int y0 = fy0 < 0.f ? 0 : (fy0 > (float)H ? H : (int)fy0);
    int y1 = fy1 > (float)(H - 1) ? H - 1 : (fy1 < -1.f ? -1 : (int)fy1);
    if (x0 > x1 || y0 > y1) return false;
    tx0 = x0 / T;
    tx1 = x1 / T;
    ty0 = y0 / T;
    ty1 = y1 / T;
    return true;
}

// Level of the alpha >= alpha_min ellipse for the tile test: ex^2 (a c - b^2) / c is
// 2 ln(o / alpha_min), the level whose bounding box has the footprint half-width ex; a
// relative margin of 1e-3 plus 1e-3 keeps the test conservative under rounding.
__device__ __forceinline__ float tile_tau2(float a, float b, float c, float ex) {
    const float det = __fsub_rn(__fmul_rn(a, c), __fmul_rn(b, b));
    const float t = __fdiv_rn(__fmul_rn(__fmul_rn(ex, ex), det), c);
    return __fadd_rn(__fmul_rn(t, 1.001f), 1e-3f);
}

// a x^2 + 2 b x y + c y^2, explicitly rounded steps.
__device__ __forceinline__ float tile_q(float a, float b, float c, float x, float y) {
    const float t1 = __fmul_rn(__fmul_rn(a, x), x);
    const float t2 = __fmul_rn(__fmul_rn(__fmul_rn(2.f, b), x), y);
    const float t3 = __fmul_rn(__fmul_rn(c, y), y);
    return __fadd_rn(__fadd_rn(t1, t2), t3);
}

// Whether the ellipse Q(d) = a dx^2 + 2 b dx dy + c dy^2 <= tau2 (d = pixel centre - (u, v))
// reaches the pixel centres of tile (tx, ty) of a W x H view: (u, v) inside the rectangle of
// those centres, a corner with Q <= tau2, or an edge whose interior holds the quadratic's
// minimiser along it with that minimum, X^2 (a c - b^2) / c for x = X, at most tau2
// (compared as X^2 det <= tau2 c: no division).  Every step is one explicitly rounded
// single-precision operation, so that the decision can be reproduced bit for bit; NaN keeps
// the tile.
__device__ __forceinline__ bool tile_reached(float u, float v, float a, float b, float c, float tau2, int tx,
                                             int ty, int T, int W, int H) {
    const float X0 = (float)(tx * T) + 0.5f;
    const float X1 = (float)((tx + 1) * T < W ? (tx + 1) * T : W) - 0.5f;
    const float Y0 = (float)(ty * T) + 0.5f;
    const float Y1 = (float)((ty + 1) * T < H ? (ty + 1) * T : H) - 0.5f;
    const float lx = __fsub_rn(X0, u), hx = __fsub_rn(X1, u), ly = __fsub_rn(Y0, v), hy = __fsub_rn(Y1, v);
    const float det = __fsub_rn(__fmul_rn(a, c), __fmul_rn(b, b));
    bool hit = lx <= 0.f && hx >= 0.f && ly <= 0.f && hy >= 0.f;
    hit |= !(tile_q(a, b, c, lx, ly) > tau2);
    hit |= !(tile_q(a, b, c, lx, hy) > tau2);
    hit |= !(tile_q(a, b, c, hx, ly) > tau2);
    hit |= !(tile_q(a, b, c, hx, hy) > tau2);
    const float tc = __fmul_rn(tau2, c), ta = __fmul_rn(tau2, a);
    const float cly = __fmul_rn(c, ly), chy = __fmul_rn(c, hy), alx = __fmul_rn(a, lx), ahx = __fmul_rn(a, hx);
    const float m0 = -__fmul_rn(b, lx), m1 = -__fmul_rn(b, hx), m2 = -__fmul_rn(b, ly), m3 = -__fmul_rn(b, hy);
    hit |= cly <= m0 && m0 <= chy && !(__fmul_rn(__fmul_rn(lx, lx), det) > tc);
    hit |= cly <= m1 && m1 <= chy && !(__fmul_rn(__fmul_rn(hx, hx), det) > tc);
    hit |= alx <= m2 && m2 <= ahx && !(__fmul_rn(__fmul_rn(ly, ly), det) > ta);
    hit |= alx <= m3 && m3 <= ahx && !(__fmul_rn(__fmul_rn(hy, hy), det) > ta);
    return hit;
}

// Real spherical harmonics (Condon-Shortley phase, l-major, m = -l..l) as polynomials in
// the unit direction; the constants are the normalisations sqrt((2l+1)/(4pi)(l-m)!/(l+m)!)
// times the sqrt(2) of the real combination, folded into each monomial.
struct SHConst {
    static constexpr float c0 = 0.28209479177387814f;   // 1/(2 sqrt(pi))
    static constexpr float c1 = 0.48860251190291992f;   // sqrt(3/(4 pi))
    static constexpr float c2a = 1.0925484305920792f;   // sqrt(15/pi)/2
    static constexpr float c2b = 0.31539156525252005f;  // sqrt(5/pi)/4
    static constexpr float c2c = 0.54627421529603959f;  // sqrt(15/pi)/4
    static constexpr float c3a = 0.59004358992664352f;  // sqrt(35/(2 pi))/4
    static constexpr float c3b = 2.8906114426405538f;   // sqrt(105/pi)/2
    static constexpr float c3c = 0.45704579946446572f;  // sqrt(21/(2 pi))/4
    static constexpr float c3d = 0.37317633259011540f;  // sqrt(7/pi)/4
    static constexpr float c3e = 1.4453057213202769f;   // sqrt(105/pi)/4
};

__device__ __forceinline__ void sh_basis(int deg, float x, float y, float z, float* Y) {
    Y[0] = SHConst::c0;
    if (deg < 1) return;
    Y[1] = -SHConst::c1 * y;
    Y[2] = SHConst::c1 * z;
    Y[3] = -SHConst::c1 * x;
    if (deg < 2) return;
    float xx = x * x, yy = y * y, zz = z * z;
    Y[4] = SHConst::c2a * x * y;
    Y[5] = -SHConst::c2a * y * z;
    Y[6] = SHConst::c2b * (2.f * zz - xx - yy);
    Y[7] = -SHConst::c2a * x * z;
    Y[8] = SHConst::c2c * (xx - yy);
    if (deg < 3) return;
    Y[9] = -SHConst::c3a * y * (3.f * xx - yy);
    Y[10] = SHConst::c3b * x * y * z;
    Y[11] = -SHConst::c3c * y * (4.f * zz - xx - yy);
    Y[12] = SHConst::c3d * z * (2.f * zz - 3.f * xx - 3.f * yy);
    Y[13] = -SHConst::c3c * x * (4.f * zz - xx - yy);
    Y[14] = SHConst::c3e * z * (xx - yy);
    Y[15] = -SHConst::c3a * x * (xx - 3.f * yy);
}

// Gradient of each basis polynomial with respect to (x, y, z): dY[k][0..2].
__device__ __forceinline__ void sh_basis_grad(int deg, float x, float y, float z, float (*dY)[3]) {
    dY[0][0] = dY[0][1] = dY[0][2] = 0.f;
    if (deg < 1) return;
    dY[1][0] = 0.f; dY[1][1] = -SHConst::c1; dY[1][2] = 0.f;
    dY[2][0] = 0.f; dY[2][1] = 0.f; dY[2][2] = SHConst::c1;
    dY[3][0] = -SHConst::c1; dY[3][1] = 0.f; dY[3][2] = 0.f;
    if (deg < 2) return;
    float xx = x * x, yy = y * y, zz = z * z;
    dY[4][0] = SHConst::c2a * y; dY[4][1] = SHConst::c2a * x; dY[4][2] = 0.f;
    dY[5][0] = 0.f; dY[5][1] = -SHConst::c2a * z; dY[5][2] = -SHConst::c2a * y;
    dY[6][0] = -2.f * SHConst::c2b * x; dY[6][1] = -2.f * SHConst::c2b * y; dY[6][2] = 4.f * SHConst::c2b * z;
    dY[7][0] = -SHConst::c2a * z; dY[7][1] = 0.f; dY[7][2] = -SHConst::c2a * x;
    dY[8][0] = 2.f * SHConst::c2c * x; dY[8][1] = -2.f * SHConst::c2c * y; dY[8][2] = 0.f;
    if (deg < 3) return;
    dY[9][0] = -6.f * SHConst::c3a * x * y;
    dY[9][1] = -SHConst::c3a * (3.f * xx - 3.f * yy);
    dY[9][2] = 0.f;
    dY[10][0] = SHConst::c3b * y * z; dY[10][1] = SHConst::c3b * x * z; dY[10][2] = SHConst::c3b * x * y;
    dY[11][0] = 2.f * SHConst::c3c * x * y;
    dY[11][1] = -SHConst::c3c * (4.f * zz - xx - 3.f * yy);
    dY[11][2] = -8.f * SHConst::c3c * y * z;
    dY[12][0] = -6.f * SHConst::c3d * x * z;
    dY[12][1] = -6.f * SHConst::c3d * y * z;
    dY[12][2] = SHConst::c3d * (6.f * zz - 3.f * xx - 3.f * yy);
    dY[13][0] = -SHConst::c3c * (4.f * zz - 3.f * xx - yy);
    dY[13][1] = 2.f * SHConst::c3c * x * y;
    dY[13][2] = -8.f * SHConst::c3c * x * z;
    dY[14][0] = 2.f * SHConst::c3e * x * z; dY[14][1] = -2.f * SHConst::c3e * y * z;
    dY[14][2] = SHConst::c3e * (xx - yy);
    dY[15][0] = -SHConst::c3a * (3.f * xx - 3.f * yy);
    dY[15][1] = 6.f * SHConst::c3a * x * y;
    dY[15][2] = 0.f;
}

// sum_k w[k] grad Y_k(x, y, z) for k >= 1, without materialising the 16 x 3 Jacobian.
__device__ __forceinline__ void sh_grad_dot(int deg, float x, float y, float z, const float* w, float* g) {
    g[0] = g[1] = g[2] = 0.f;
    if (deg < 1) return;
    g[0] += -SHConst::c1 * w[3];
    g[1] += -SHConst::c1 * w[1];
    g[2] += SHConst::c1 * w[2];
    if (deg < 2) return;
    const float xx = x * x, yy = y * y, zz = z * z;
    g[0] += SHConst::c2a * (y * w[4] - z * w[7]) + SHConst::c2b * (-2.f * x) * w[6] + 2.f * SHConst::c2c * x * w[8];
    g[1] += SHConst::c2a * (x * w[4] - z * w[5]) + SHConst::c2b * (-2.f * y) * w[6] - 2.f * SHConst::c2c * y * w[8];
    g[2] += -SHConst::c2a * (y * w[5] + x * w[7]) + 4.f * SHConst::c2b * z * w[6];
    if (deg < 3) return;
    g[0] += -6.f * SHConst::c3a * x * y * w[9] + SHConst::c3b * y * z * w[10] +
            2.f * SHConst::c3c * x * y * w[11] - 6.f * SHConst::c3d * x * z * w[12] -
            SHConst::c3c * (4.f * zz - 3.f * xx - yy) * w[13] + 2.f * SHConst::c3e * x * z * w[14] -
            SHConst::c3a * (3.f * xx - 3.f * yy) * w[15];
    g[1] += -SHConst::c3a * (3.f * xx - 3.f * yy) * w[9] + SHConst::c3b * x * z * w[10] -
            SHConst::c3c * (4.f * zz - xx - 3.f * yy) * w[11] - 6.f * SHConst::c3d * y * z * w[12] +
            2.f * SHConst::c3c * x * y * w[13] - 2.f * SHConst::c3e * y * z * w[14] +
            6.f * SHConst::c3a * x * y * w[15];
    g[2] += SHConst::c3b * x * y * w[10] - 8.f * SHConst::c3c * y * z * w[11] +
            SHConst::c3d * (6.f * zz - 3.f * xx - 3.f * yy) * w[12] - 8.f * SHConst::c3c * x * z * w[13] +
            SHConst::c3e * (xx - yy) * w[14];
}

// Row r of a structure-of-arrays buffer with n columns: a wave-uniform base pointer, so
// per-lane accesses need only the 32-bit lane offset.
template <typename T>
__device__ __forceinline__ T* sh_row(T* base, int n, int r) {
    return base + (size_t)r * (size_t)n;
}

// Returns p unchanged but opaque to the optimiser (an empty asm on a scalar register), so
// addresses derived from it inside a loop are not hoisted into long-lived vector registers.
template <typename T>
__device__ __forceinline__ T* opaque_ptr(T* p) {
    asm volatile("" : "+s"(p));
    return p;
}

// Unit quaternion (w, x, y, z) -> row-major rotation matrix.
// World -> camera point x_c = R mu + t of camera `cam`, evaluated in float64 and rounded
// once.  Far from the frame origin (one global map, sub-maps hundreds of metres apart) R mu
// and t nearly cancel, and a float32 evaluation would keep only |t| 2^-24 (1e-4 m at 1.4 km)
// of the metre-scale difference; each float32 x float32 product is exact in float64.
__device__ __forceinline__ void world_to_cam(const ags_camera& cam, float mx, float my, float mz, float& x,
                                             float& y, float& z) {
    const double X = mx, Y = my, Z = mz;
    const float* R = cam.R;
    x = (float)fma((double)R[0], X, fma((double)R[1], Y, fma((double)R[2], Z, (double)cam.t[0])));
    y = (float)fma((double)R[3], X, fma((double)R[4], Y, fma((double)R[5], Z, (double)cam.t[1])));
    z = (float)fma((double)R[6], X, fma((double)R[7], Y, fma((double)R[8], Z, (double)cam.t[2])));
}

// mu - C, the vector from camera `cam`'s centre C = -R^T t to the mean (the SH viewing
// direction before normalisation), in float64 for the same reason.
__device__ __forceinline__ void centre_to_mean(const ags_camera& cam, float mx, float my, float mz, float& dx,
                                               float& dy, float& dz) {
    const double t0 = cam.t[0], t1 = cam.t[1], t2 = cam.t[2];
    const float* R = cam.R;
    dx = (float)fma((double)R[0], t0, fma((double)R[3], t1, fma((double)R[6], t2, (double)mx)));
    dy = (float)fma((double)R[1], t0, fma((double)R[4], t1, fma((double)R[7], t2, (double)my)));
    dz = (float)fma((double)R[2], t0, fma((double)R[5], t1, fma((double)R[8], t2, (double)mz)));
}

__device__ __forceinline__ void quat_to_rot(float w, float x, float y, float z, float* R) {
    R[0] = 1.f - 2.f * (y * y + z * z); R[1] = 2.f * (x * y - w * z); R[2] = 2.f * (x * z + w * y);
    R[3] = 2.f * (x * y + w * z); R[4] = 1.f - 2.f * (x * x + z * z); R[5] = 2.f * (y * z - w * x);
    R[6] = 2.f * (x * z - w * y); R[7] = 2.f * (y * z + w * x); R[8] = 1.f - 2.f * (x * x + y * y);
}

// Wave-wide sum of one float (64 lanes); every lane gets the total.

__device__ __forceinline__ unsigned lane_id() { return __lane_id(); }

// Sum of 16 per-lane values over the 64-lane wave (a transposing butterfly).  On return
// lane L holds the total of slot (L >> 2) & 15.  Each stage pairs lanes that differ in one
// selector bit; a lane keeps the half of its slots named by that bit and adds the
// partner's copy of the same half.  Bits 5 and 4 use the gfx950 lane-swap instructions
// (v_permlane32_swap / v_permlane16_swap exchange exactly those halves, so keep + partner
// is result[0] + result[1] on every lane); bits 3 and 2 use DPP row_ror:8 and
// row_half_mirror (involutions pairing lanes that differ in that bit); bits 1 and 0 are
// quad permutations.
template <int CTRL>
__device__ __forceinline__ float dpp_mov(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}

// Sum over the 64-lane wave, returned in every lane: lane halves and row pairs through the
// gfx950 lane swaps, then rotations inside each 16-lane row.
__device__ __forceinline__ float wave_sum(float v) {
    auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(v), __float_as_uint(v), false, false);
    v = __uint_as_float(r[0]) + __uint_as_float(r[1]);
    r = __builtin_amdgcn_permlane16_swap(__float_as_uint(v), __float_as_uint(v), false, false);
    v = __uint_as_float(r[0]) + __uint_as_float(r[1]);
    v += dpp_mov<0x128>(v);  // row_ror:8
    v += dpp_mov<0x124>(v);  // row_ror:4
    v += dpp_mov<0x122>(v);  // row_ror:2
    v += dpp_mov<0x121>(v);  // row_ror:1
    return v;
}

__device__ __forceinline__ float wave_transpose_sum16(const float (&v)[16]) {
    const int lane = __lane_id();
    float w8[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(v[j]), __float_as_uint(v[j + 8]), false,
                                                  false);
        w8[j] = __uint_as_float(r[0]) + __uint_as_float(r[1]);
    }
    float w4[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(w8[j]), __float_as_uint(w8[j + 4]), false,
                                                  false);
        w4[j] = __uint_as_float(r[0]) + __uint_as_float(r[1]);
    }
    float w2[2];
    {
        const bool hi = lane & 8;
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const float send = hi ? w4[j] : w4[j + 2];
            const float keep = hi ? w4[j + 2] : w4[j];
            w2[j] = keep + dpp_mov<0x128>(send);  // row_ror:8 == lane ^ 8 inside a row
        }
    }
    float w1;
    {
        const bool hi = lane & 4;
        const float send = hi ? w2[0] : w2[1];
        const float keep = hi ? w2[1] : w2[0];
        w1 = keep + dpp_mov<0x141>(send);  // row_half_mirror: lane i <-> 7 - i in 8-lane halves
    }
    w1 += dpp_mov<0xB1>(w1);  // quad_perm [1, 0, 3, 2]: lane ^ 1
    w1 += dpp_mov<0x4E>(w1);  // quad_perm [2, 3, 0, 1]: lane ^ 2
    return w1;
}

// Sum of 10 per-lane values over the wave with the same butterfly, the values placed in
// slots {0, 1, 2, 4, 5} (v < 5) and {8, 9, 10, 12, 13} (v >= 5) so that no stage pairs two
// empty slots: 5 + 3 lane swaps, then 3 DPP stages.  Lanes of empty slots end with
// meaningless sums (only empty-slot data flows into them).  On return lane L holds the
// total of slot (L >> 2) & 15.
__device__ __forceinline__ float wave_transpose_sum10(const float (&v)[10]) {
    const int lane = __lane_id();
    // stage 1 (lane bit 5): value j and j + 5 share slot low bits kSlot[j] = {0, 1, 2, 4, 5}
    float w8[5];
#pragma unroll
    for (int j = 0; j < 5; ++j) {
        auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(v[j]), __float_as_uint(v[j + 5]), false,
                                                  false);
        w8[j] = __uint_as_float(r[0]) + __uint_as_float(r[1]);
    }
    // stage 2 (lane bit 4): slot low bits (0, 4) -> w8[0], w8[3]; (1, 5) -> w8[1], w8[4];
    // (2, 6) -> w8[2] and an empty slot
    float w4[3];
    {
        auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(w8[0]), __float_as_uint(w8[3]), false, false);
        w4[0] = __uint_as_float(r[0]) + __uint_as_float(r[1]);
        r = __builtin_amdgcn_permlane16_swap(__float_as_uint(w8[1]), __float_as_uint(w8[4]), false, false);
        w4[1] = __uint_as_float(r[0]) + __uint_as_float(r[1]);
        r = __builtin_amdgcn_permlane16_swap(__float_as_uint(w8[2]), __float_as_uint(w8[2]), false, false);
        w4[2] = __uint_as_float(r[0]) + __uint_as_float(r[1]);
    }
    // stage 3 (lane bit 3): (w4[0], w4[2]); w4[1]'s partner slot is empty, so both lane
    // halves simply add their neighbour's w4[1]
    float w2[2];
    {
        const bool hi = lane & 8;
        const float send = hi ? w4[0] : w4[2];
        const float keep = hi ? w4[2] : w4[0];
        w2[0] = keep + dpp_mov<0x128>(send);  // row_ror:8 == lane ^ 8 inside a row
        w2[1] = w4[1] + dpp_mov<0x128>(w4[1]);
    }
    // stage 4 (lane bit 2), then lane bits 0 and 1
    float w1;
    {
        const bool hi = lane & 4;
        const float send = hi ? w2[0] : w2[1];
        const float keep = hi ? w2[1] : w2[0];
        w1 = keep + dpp_mov<0x141>(send);  // row_half_mirror: lane i <-> 7 - i in 8-lane halves
    }
    w1 += dpp_mov<0xB1>(w1);  // quad_perm [1, 0, 3, 2]: lane ^ 1
    w1 += dpp_mov<0x4E>(w1);  // quad_perm [2, 3, 0, 1]: lane ^ 2
    asm volatile("" : "+v"(w1));  // the last step stays one DPP add, ahead of the caller's branch
    return w1;
}

// Host-side launchers (one per kernel family), defined next to their kernels.
struct ProjectArgs {
    ViewTable vt;
    Settings st;
    int n, sh_degree;
    const float *means, *log_scales, *quats, *logits, *sh;
    const ags_camera* cams;
    float* records;
    uint32_t* pair_count;
    uint32_t* pair_z;
    float* grad2d;  // [n_pairs][kGrad2dStride]: each visible pair's row is zeroed for the backward
};
void launch_project_fwd(const ProjectArgs& a, hipStream_t s);

void launch_fill_u32(uint32_t* p, uint32_t v, long long n, hipStream_t s);
void launch_fill_f32(float* p, float v, long long n, hipStream_t s);

// Exclusive scan of n u32 values (n read from device if n_dev != nullptr, else n_max).
// Value source: src[i], or src[idx[i]] when idx != nullptr, or (src[i] != 0) when
// as_flags.  Writes out[i] and total to *total (if non-null).
struct ScanTemp {
    uint32_t* block_sums;   // >= scan_blocks(n_max)
};
long long scan_blocks(long long n_max);
void launch_scan(const uint32_t* src, const uint32_t* idx, bool as_flags, uint32_t* out,
                 long long n_max, const uint32_t* n_dev, uint32_t* total, ScanTemp tmp,
                 hipStream_t s);

// Depth key of a (view, Gaussian) pair that no tile receives: a NaN bit pattern, never the
// bits of a depth >= z_near.
constexpr uint32_t kNoDepth = 0xFFFFFFFFu;

// Output slots per emission workgroup.
constexpr int kEmitSlots = 512;

// Exclusive scan of counts[order[i]] (counts[i] when order is null; out may then be
// counts itself) over i < *n_dev into out, for the intersection
// emission: also sets counters[CNT_K / CNT_OVERFLOW / CNT_KEFF] against `capacity` and, for
// each kEmitSlots-slot emission workgroup below capacity, the item owning its first slot.
void launch_emit_scan(const uint32_t* counts, const uint32_t* order, uint32_t* out, long long n_max,
                      const uint32_t* n_dev, uint32_t* counters, long long capacity, uint32_t* block_first,
                      ScanTemp tmp, hipStream_t s);

// Stable LSD radix sort of (key, value) u32 pairs on bits [0, bits), n read from n_dev,
// with `grid` workgroups per pass (sort_grid of the static maximum, at most 256).
struct SortTemp {
    uint32_t* hist;         // sort_hist_entries(grid): per-workgroup digit totals, then offsets
    uint32_t* rowtot;       // sort_rowtot_entries(): per-digit totals
};
int sort_grid(long long n_max);
int sort_passes(int bits);
long long sort_hist_entries(int grid);
long long sort_rowtot_entries();
// keys/vals: [0] = input, [1] = other buffer; returns index of the buffer holding the
// result (0 or 1).  With gather_out, the last pass also writes gather_out[i] =
// gather_src[sorted value i].  With n_live, the first pass drops the items whose key is
// drop_key, writes how many are kept to *n_live, and the later passes sort only those.
// With first_keys, the first pass reads its keys from there and takes each item's index as
// its value (keys[0] / vals[0] are then only written); the result is in buffer
// (passes - 1) % 2.
int launch_radix_sort(uint32_t* keys[2], uint32_t* vals[2], long long n_max, const uint32_t* n_dev,
                      int bits, int grid, SortTemp tmp, hipStream_t s, const uint32_t* gather_src = nullptr,
                      uint32_t* gather_out = nullptr, uint32_t* n_live = nullptr, uint32_t drop_key = 0u,
                      const uint32_t* first_keys = nullptr);

struct BinArgs {
    ViewTable vt;
    const float* records;
    const uint32_t* pair_count;
    const uint32_t* pair_z;
    uint32_t* counters;
    long long n_pairs;
    long long capacity;
    uint32_t* depth_keys[2]; // [n_pairs]
    uint32_t* depth_vals[2];
    uint32_t* emit_off;      // [n_pairs] scan of tile counts in depth order
    uint32_t* block_first;   // [capacity / kEmitSlots + 1] first depth-ordered pair of each emit workgroup
    uint32_t* tile_keys[2];  // [capacity]
    uint32_t* tile_vals[2];
    uint32_t* ranges;        // [n_tiles][2]
    uint32_t* work;          // [n_tiles] raster work order: tiles by descending list length
    uint32_t* final_vals;    // where the tile-sorted pair ids must end (== one of tile_vals)
    int tile_bits;
    ScanTemp scan_tmp;
    SortTemp sort_tmp;
    int depth_grid, tile_grid;  // radix-sort workgroups of the two sorts
};
void launch_count_from_records(const ViewTable& vt, const float* records, const uint8_t* valid,
                               long long n_pairs, uint32_t* pair_count, uint32_t* pair_z,
                               hipStream_t s);
// Runs the depth sort (its first pass drops the pairs no tile receives), tile-count scan,
// emission, tile sort and ranges.  Returns 0 or a HIP error.
int launch_binning(BinArgs& a, hipStream_t s);

struct RasterArgs {
    ViewTable vt;
    Settings st;
    const float* records;
    const uint32_t* tile_pairs;
    const uint32_t* ranges;
    const uint32_t* work;  // [n_tiles] tile of each workgroup, longest lists first
    float* rgb;
    float* depth;
    float* alpha;
    float* depth_var;  // or null: rendered depth variance per pixel
    float* t_final;
    uint32_t* last;
    // zeroed per pixel (or null): the backward's dense depth and second-moment adjoints
    float* zero_px[2];
};
// The (tile, pixels per thread, LDS batch) launch shapes compiled for both raster kernels:
// writes up to n_max of them and returns how many there are.
int raster_shapes(int* tile, int* ppt, int* batch, int n_max);
int launch_raster_fwd(const RasterArgs& a, int T, int batch, int ppt, hipStream_t s);

struct RasterBwdArgs {
    ViewTable vt;
    Settings st;
    const float* records;
    const uint32_t* tile_pairs;
    const uint32_t* ranges;
    const uint32_t* work;  // as in RasterArgs
    const float* t_final;
    const uint32_t* last;
    // upstream mode
    const float* d_rgb;
    const float* d_depth;
    const float* d_alpha;
    // loss mode (fused L1 prologue); d_depth then points at the scattered LiDAR adjoint and
    // d_rgb (or null) at the adjoint of the D-SSIM part, both added to the pixel's adjoints;
    // d_depth2 (or null) at the LiDAR adjoint of the second depth moment (rendered variance)
    int loss_mode;
    const float* d_depth2;
    const float* rgb;
    const float* gt_rgb;
    const uint8_t* mask;
    float l1_scale[kMaxViews];   // (1 - lambda_ssim) w_l1 / (3 n_b)
    float* loss_partials;        // one per block (loss mode)
    float* grad2d;               // [n_pairs][16] (ten used); rows of visible pairs cleared
};
int launch_raster_bwd(const RasterBwdArgs& a, int T, int batch, int ppt, hipStream_t s);
// The backward's clears in one launch, for a backward whose forward did not leave them done
// (a second backward of one forward): grad2d's rows of the pairs with pair_count != 0 (the
// rows raster_bwd adds to; none if grad2d is null), and up to kBwdClearRegions float buffers
// (the dense depth adjoints; zero_n[r] floats each, 0 for none).
constexpr int kBwdClearRegions = 2;
struct BwdClearArgs {
    float* grad2d;
    const uint32_t* pair_count;
    long long n_pairs;
    float* zero[kBwdClearRegions];
    long long zero_n[kBwdClearRegions];
};
void launch_bwd_clear(const BwdClearArgs& a, hipStream_t s);
int raster_blocks(const ViewTable& vt);
// Raster work list: strips of kWorkStrip consecutive tiles go round-robin to the eight XCDs
// (workgroup g runs on XCD g % 8); each XCD takes its strips' tiles longest list first.
// raster_blocks() workgroups, some of them (at most 8 (kWorkStrip + 1)) with no tile.
constexpr int kWorkStrip = 8;
constexpr uint32_t kNoTile = 0xFFFFFFFFu;

struct SsimArgs {
    ViewTable vt;
    const float* rgb;            // rendered colour (rgb layout)
    const float* gt_rgb;         // target colour (rgb layout)
    const uint8_t* mask;         // [P] or null
    float scale[kMaxViews];      // lambda w_l1 / (3 n_b)
    float* d_rgb;                // out: adjoint of the D-SSIM part (rgb layout)
    float* partials;             // out: one loss partial per workgroup (ssim_blocks)
    int tile_base[kMaxViews + 1];  // filled by the launcher
    float w[11];                   // window weights, filled by the launcher
};
long long ssim_blocks(const ViewTable& vt);
void launch_ssim(SsimArgs a, hipStream_t s);

struct LidarArgs {
    ViewTable vt;
    const float* depth;
    const float* depth_var;      // rendered variance mode: rendered depth variance, else null
    float sigma_floor;
    float* d_depth2;             // rendered variance mode: dense [P] adjoint (zeroed before)
    const int32_t* pix;
    const float* val;
    const float* sigma;
    long long n_targets;
    long long target_off[kMaxViews + 1];
    float scale[kMaxViews];      // lambda / |Omega_b|
    float* d_depth;              // dense [P] (zeroed before)
    float* loss_partials;
};
int lidar_blocks(long long n_targets);
void launch_lidar_adjoint(const LidarArgs& a, hipStream_t s);
void launch_sum_partials(const float* partials, long long n, long long skip0, long long skip1, float* out,
                         hipStream_t s);

// Adam on the Gaussian parameters: groups means, log-scales, quaternions, logits, SH
// degree 0, SH degree >= 1 (lr[0..5]); the SH buffer holds both SH groups.
struct AdamArgs {
    int n, sh_k;
    float* p[5];
    const float* g[5];
    float* m[5];
    float* v[5];
    float lr[6];
    float beta1, beta2, eps;
    const int32_t* step;
};

// One Adam update of one value (torch.optim.Adam without weight decay); bc1, bc2 are the
// bias corrections 1 - beta^t.  The moment updates are written as explicit fused
// multiply-adds so every kernel that inlines this rounds them the same way.
__device__ __forceinline__ void adam_one(float& p, float g, float& m, float& v, float lr, float b1, float b2,
                                         float bc1, float bc2, float eps) {
    m = fmaf(b1, m, (1.f - b1) * g);
    v = fmaf(b2, v, ((1.f - b2) * g) * g);
    p -= lr * (m / bc1) / (sqrtf(v / bc2) + eps);
}

struct ProjectBwdArgs {
    ViewTable vt;
    Settings st;
    int n, sh_degree;
    const float *means, *log_scales, *quats, *logits, *sh;
    const ags_camera* cams;
    const uint32_t* pair_count;
    const float* records;   // the forward's records (stored colour: the clamp mask)
    const float* grad2d;
    float *g_means, *g_log_scales, *g_quats, *g_logits, *g_sh, *g_pose;
    float* pose_partials;  // [n_views * 6][2 project_bwd_blocks(n)]: geometry, then colour
    uint32_t* vis_mask;    // [n]: views keeping each Gaussian (geometry phase -> colour phase)
    float* stat_grad;      // [n] or null: += |dL/d(u, v)| per view seeing the Gaussian
    float* stat_count;     // [n] or null: += number of those views
    int accumulate;
    // fused optimiser step: the colour phase, which finishes each Gaussian's gradient, applies
    // Adam to all its parameters instead of writing the SH gradient (g_sh unused)
    int fused_adam;
    AdamArgs adam;
    // optional (loss_out non-null): the loss partials' fixed-order sum into loss_out[0], done
    // by one more workgroup of the pose reduction's launch; entries [loss_skip0, loss_skip1)
    // were not written and count as zero
    const float* loss_partials;
    long long n_loss, loss_skip0, loss_skip1;
    float* loss_out;
};
int project_bwd_blocks(int n);
void launch_project_bwd(const ProjectBwdArgs& a, hipStream_t s);

struct LifecycleArgs {
    int n, k3;                     // inputs, SH floats per Gaussian (3 K)
    int chunks;                    // scatter launch rows per array (set by launch_lifecycle)
    long long cap;                 // output capacity (row stride of the outputs)
    const float* in[3][5];         // [params, m, v][means, log_scales, quats, logits, sh]
    float* out[3][5];
    const float* stat_grad;
    const float* stat_count;
    const float* noise;            // [n][2][3]
    int do_prune, do_densify, do_reset;
    float tau_opa, s_min, s_max, grad_threshold, kappa, two_s_init, tau_reset;
    float reset_logit, log_split;
    uint32_t* counts;              // [n] outputs per input (scratch)
    uint32_t* offsets;             // [n] first output slot (scratch)
    uint8_t* actions;              // [n] or null
    int32_t* n_out;
    ScanTemp scan_tmp;
};
void launch_lifecycle(const LifecycleArgs& a, hipStream_t s);
// Device address and size of the lifecycle pass's static scratch array on `device` (looked
// up on the first call for that device, with the device made current meanwhile).
int lifecycle_static_scratch(int device, void** ptr, size_t* bytes);

// Profiled stages (ags_profile_read reports their times under these indices).
enum Stage {
    ST_PROJECT = 0,
    ST_BINNING,
    ST_RASTER_FWD,
    ST_LIDAR,
    ST_RASTER_BWD,
    ST_PROJECT_BWD,
    ST_CLEAR,
    ST_ADAM,
    ST_POSE,
    ST_SSIM,
    ST_LIFECYCLE,
    ST_MAP_PROBE,
    ST_MAP_LRU,
    ST_MAP_REBUILD,
    ST_MAP_COPY,
    ST_COUNT
};

// Brackets a group of launches on stream s with events while the context profiles.
struct StageTimer {
    ags_ctx* ctx;
    int stage;
    hipStream_t s;
    hipEvent_t a = nullptr, b = nullptr;
    StageTimer(ags_ctx* c, int st, hipStream_t str);
    ~StageTimer();
    hipEvent_t take();
};

// Context access for sources other than the context's own: its device, and recording a
// failed HIP call (returns AGS_ERR_HIP).
int ctx_device(const ags_ctx* ctx);
int ctx_record_hip(ags_ctx* ctx, hipError_t e);

void launch_adam(const AdamArgs& a, hipStream_t s);
void launch_count_nonfinite(const float* x, long long n, int32_t* bad, hipStream_t s);
void launch_pose_step(ags_camera* cams, int n_views, const float* g, float* m, float* v,
                      int32_t* step, int advance, float lr, float b1, float b2, float eps,
                      hipStream_t s);

}  // namespace ags
