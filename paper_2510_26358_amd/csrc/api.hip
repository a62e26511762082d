// C ABI of libagsplat: argument validation, buffer layout and launch sequencing.
// Kernels live in the other translation units; this file only enqueues them.
#include <math.h>
#include <string.h>

#include <new>
#include <vector>

#include "common.h"

using namespace ags;

struct ProfEvent {
    int stage;
    hipEvent_t a, b;
};

static const char* kStageNames[ST_COUNT] = {"project_fwd", "binning",     "raster_fwd",
                                             "lidar_adjoint", "raster_bwd", "project_bwd",
                                             "clear",       "adam",        "pose_step", "ssim",
                                             "lifecycle",   "map_probe",   "map_lru",   "map_rebuild",
                                             "map_copy"};

struct ags_ctx {
    int device;
    ags_config cfg;
    void* static_scratch;      // device address of the lifecycle pass's static scratch
    size_t static_scratch_bytes;
    int last_hip;
    bool prof;
    std::vector<ProfEvent> pending;
    std::vector<hipEvent_t> pool;
    double total_ms[ST_COUNT];
    long long launches[ST_COUNT];
    // What the last forward call on this context left zeroed in its `saved`
    // buffer for the backward: the visible pairs' adjoint rows (kClearRows), the dense depth
    // adjoint (kClearDepth) and second-moment adjoint (kClearDepth2); recorded with the
    // stream capture it was enqueued in (0: none).  A backward of the same buffer in the same
    // capture state skips those clears and resets the record, since it dirties them.
    const void* clean_saved;
    unsigned clean_bits;
    unsigned long long clean_capture;
};

namespace {

constexpr size_t kAlign = 256;
size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }
// the kernels read records and sorted keys as 16-byte vectors at offsets that are multiples
// of kAlign from the buffer's start
bool misaligned(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) != 0; }

struct Layout {
    ViewTable vt;
    long long Q, P, n_tiles, cap;
    int tile_bits;
    int depth_grid, tile_grid;
    // saved
    size_t s_counters, s_records, s_pair_count, s_tile_pairs, s_ranges, s_work, s_t_final, s_last, s_grad2d,
        s_ddepth, s_ddepth2, s_total;
    // fwd ws
    size_t f_pair_z, f_dkeys0, f_dkeys1, f_dvals0, f_dvals1, f_emit_off, f_block_first, f_tkeys0, f_tkeys1,
        f_tvals1, f_hist, f_rowtot, f_block_sums, f_total;
    // bwd ws
    size_t b_dssim, b_partials, b_pose_part, b_vis, b_total;
    long long n_partials, n_ssim;
};

int check_views(const ags_views* v) {
    if (!v || v->n_views < 1 || v->n_views > AGS_MAX_VIEWS) return AGS_ERR_INVALID_ARG;
    if (!v->width || !v->height || !v->g_begin || !v->g_end) return AGS_ERR_INVALID_ARG;
    return AGS_OK;
}

int check_config(const ags_config* c) {
    if (!c) return AGS_ERR_INVALID_ARG;
    if (c->tile != 8 && c->tile != 16 && c->tile != 32) return AGS_ERR_INVALID_ARG;
    if (c->batch != 64 && c->batch != 128 && c->batch != 256 && c->batch != 512) return AGS_ERR_INVALID_ARG;
    if (c->px_per_thread != 1 && c->px_per_thread != 2 && c->px_per_thread != 4) return AGS_ERR_INVALID_ARG;
    if (c->batch_bwd != 0 && c->batch_bwd != 64 && c->batch_bwd != 128 && c->batch_bwd != 256 &&
        c->batch_bwd != 512)
        return AGS_ERR_INVALID_ARG;
    if (c->px_per_thread_bwd != 0 && c->px_per_thread_bwd != 1 && c->px_per_thread_bwd != 2 &&
        c->px_per_thread_bwd != 4)
        return AGS_ERR_INVALID_ARG;
    if (!(c->alpha_min > 0.f && c->alpha_min < c->alpha_max && c->alpha_max < 1.f)) return AGS_ERR_INVALID_ARG;
    if (!(c->t_min > 0.f && c->t_min < 1.f) || !(c->blur >= 0.f) || !(c->z_near > 0.f) ||
        !(c->fov_clamp > 0.f))
        return AGS_ERR_INVALID_ARG;
    return AGS_OK;
}

int build_layout(const ags_config* cfg, const ags_views* views, int n, long long cap, Layout& L) {
    int rc = check_views(views);
    if (rc) return rc;
    if (n < 0 || cap < 0 || cap > 0x7fffffffLL) return AGS_ERR_INVALID_ARG;
    memset(&L, 0, sizeof(L));
    ViewTable& vt = L.vt;
    vt.n_views = views->n_views;
    vt.tile = cfg->tile;
    const int T = cfg->tile;
    long long pix = 0, pair = 0, tiles = 0;
    for (int b = 0; b < views->n_views; ++b) {
        const int W = views->width[b], H = views->height[b];
        const int g0 = views->g_begin[b], g1 = views->g_end[b];
        if (W < 1 || H < 1 || W > 65535 || H > 65535) return AGS_ERR_INVALID_ARG;
        if (g0 < 0 || g1 < g0 || g1 > n) return AGS_ERR_INVALID_ARG;
        vt.width[b] = W;
        vt.height[b] = H;
        vt.g_begin[b] = g0;
        vt.g_end[b] = g1;
        vt.ntx[b] = (W + T - 1) / T;
        vt.nty[b] = (H + T - 1) / T;
        vt.tile_base[b] = (int)tiles;
        vt.pix_base[b] = pix;
        vt.pair_base[b] = pair;
        tiles += (long long)vt.ntx[b] * vt.nty[b];
        pix += (long long)W * H;
        pair += g1 - g0;
    }
    vt.tile_base[views->n_views] = (int)tiles;
    vt.pix_base[views->n_views] = pix;
    vt.pair_base[views->n_views] = pair;
    if (tiles > 0x7fffffffLL || pair > 0x7fffffffLL || pix > (1LL << 40)) return AGS_ERR_INVALID_ARG;
    L.Q = pair;
    L.P = pix;
    L.n_tiles = tiles;
    L.cap = cap;
    int bits = 0;  // tile ids 0 .. tiles - 1 and the key `tiles` of dropped intersections
    while ((1LL << bits) <= tiles) ++bits;
    L.tile_bits = bits;
    L.depth_grid = sort_grid(L.Q);
    L.tile_grid = sort_grid(L.cap);
    const long long Qs = L.Q > 0 ? L.Q : 1;
    const long long caps = L.cap > 0 ? L.cap : 1;
    size_t o = 0;
    L.s_counters = o; o = align_up(o + 64);
    L.s_records = o; o = align_up(o + (size_t)Qs * kRecFloats * 4);
    L.s_pair_count = o; o = align_up(o + (size_t)Qs * 4);
    L.s_tile_pairs = o; o = align_up(o + (size_t)caps * 4);
    L.s_ranges = o; o = align_up(o + (size_t)(tiles > 0 ? tiles : 1) * 8);
    L.s_work = o; o = align_up(o + (size_t)(tiles > 0 ? tiles + 8 * (kWorkStrip + 1) : 1) * 4);
    L.s_t_final = o; o = align_up(o + (size_t)pix * 4);
    L.s_last = o; o = align_up(o + (size_t)pix * 4);
    // the backward's accumulators, zeroed by the forward: per-pair 2D adjoint rows (the
    // visible pairs' rows, by the projection) and the dense depth and second-moment adjoints
    // (by the raster forward)
    L.s_grad2d = o; o = align_up(o + (size_t)Qs * kGrad2dStride * 4);
    L.s_ddepth = o; o = align_up(o + (size_t)(pix > 0 ? pix : 1) * 4);
    L.s_ddepth2 = o; o = align_up(o + (size_t)(pix > 0 ? pix : 1) * 4);
    L.s_total = o;
    o = 0;
    const int gmax = L.depth_grid > L.tile_grid ? L.depth_grid : L.tile_grid;
    const long long sb = scan_blocks(Qs);
    L.f_pair_z = o; o = align_up(o + (size_t)Qs * 4);
    L.f_dkeys0 = o; o = align_up(o + (size_t)Qs * 4);
    L.f_dkeys1 = o; o = align_up(o + (size_t)Qs * 4);
    L.f_dvals0 = o; o = align_up(o + (size_t)Qs * 4);
    L.f_dvals1 = o; o = align_up(o + (size_t)Qs * 4);
    L.f_emit_off = o; o = align_up(o + (size_t)Qs * 4);
    L.f_block_first = o; o = align_up(o + (size_t)(caps / kEmitSlots + 2) * 4);
    L.f_tkeys0 = o; o = align_up(o + (size_t)caps * 4);
    L.f_tkeys1 = o; o = align_up(o + (size_t)caps * 4);
    L.f_tvals1 = o; o = align_up(o + (size_t)caps * 4);
    L.f_hist = o; o = align_up(o + (size_t)sort_hist_entries(gmax) * 4);
    L.f_rowtot = o; o = align_up(o + (size_t)sort_rowtot_entries() * 4);
    L.f_block_sums = o; o = align_up(o + (size_t)sb * 4);
    L.f_total = o;
    o = 0;
    L.n_ssim = ssim_blocks(vt);
    L.n_partials = tiles + lidar_blocks(0) + L.n_ssim;  // raster, LiDAR, then D-SSIM blocks
    L.b_dssim = o; o = align_up(o + (size_t)(pix > 0 ? 3 * pix : 1) * 4);
    L.b_partials = o; o = align_up(o + (size_t)L.n_partials * 4);
    L.b_pose_part = o; o = align_up(o + (size_t)2 * (project_bwd_blocks(n) > 0 ? project_bwd_blocks(n) : 1) *
                                         views->n_views * 6 * 4);
    L.b_vis = o; o = align_up(o + (size_t)(n > 0 ? n : 1) * 4);
    L.b_total = o;
    return AGS_OK;
}

Settings settings_of(const ags_config& c) {
    Settings s;
    s.alpha_min = c.alpha_min;
    s.alpha_max = c.alpha_max;
    s.t_min = c.t_min;
    s.blur = c.blur;
    s.z_near = c.z_near;
    s.fov_clamp = c.fov_clamp;
    s.bg0 = c.bg[0];
    s.bg1 = c.bg[1];
    s.bg2 = c.bg[2];
    return s;
}

template <typename T>
T* at(void* base, size_t off) {
    return reinterpret_cast<T*>(reinterpret_cast<char*>(base) + off);
}
template <typename T>
const T* at(const void* base, size_t off) {
    return reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + off);
}

using Scope = StageTimer;

int hip_status(ags_ctx* ctx) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        if (ctx) ctx->last_hip = (int)e;
        return AGS_ERR_HIP;
    }
    return AGS_OK;
}

int check_gaussians(const ags_gaussians* g) {
    if (!g || g->n < 0 || g->sh_degree < 0 || g->sh_degree > 3) return AGS_ERR_INVALID_ARG;
    if (g->n > 0 && (!g->means || !g->log_scales || !g->quats || !g->opacity_logits || !g->sh))
        return AGS_ERR_INVALID_ARG;
    return AGS_OK;
}

BinArgs bin_args(const Layout& L, void* saved, void* ws) {
    BinArgs a;
    a.vt = L.vt;
    a.records = at<float>(saved, L.s_records);
    a.pair_count = at<uint32_t>(saved, L.s_pair_count);
    a.pair_z = at<uint32_t>(ws, L.f_pair_z);
    a.counters = at<uint32_t>(saved, L.s_counters);
    a.n_pairs = L.Q;
    a.capacity = L.cap;
    a.depth_keys[0] = at<uint32_t>(ws, L.f_dkeys0);
    a.depth_keys[1] = at<uint32_t>(ws, L.f_dkeys1);
    a.depth_vals[0] = at<uint32_t>(ws, L.f_dvals0);
    a.depth_vals[1] = at<uint32_t>(ws, L.f_dvals1);
    a.emit_off = at<uint32_t>(ws, L.f_emit_off);
    a.block_first = at<uint32_t>(ws, L.f_block_first);
    a.tile_keys[0] = at<uint32_t>(ws, L.f_tkeys0);
    a.tile_keys[1] = at<uint32_t>(ws, L.f_tkeys1);
    a.tile_vals[0] = at<uint32_t>(saved, L.s_tile_pairs);
    a.tile_vals[1] = at<uint32_t>(ws, L.f_tvals1);
    a.ranges = at<uint32_t>(saved, L.s_ranges);
    a.work = at<uint32_t>(saved, L.s_work);
    a.final_vals = a.tile_vals[0];
    a.tile_bits = L.tile_bits;
    a.scan_tmp.block_sums = at<uint32_t>(ws, L.f_block_sums);
    a.sort_tmp.hist = at<uint32_t>(ws, L.f_hist);
    a.sort_tmp.rowtot = at<uint32_t>(ws, L.f_rowtot);
    a.depth_grid = L.depth_grid;
    a.tile_grid = L.tile_grid;
    return a;
}

int run_binning(BinArgs a, hipStream_t s) { return launch_binning(a, s); }

constexpr unsigned kClearRows = 1u, kClearDepth = 2u, kClearDepth2 = 4u;

// The stream capture `s` is recording into (0: none); false if that cannot be told.  Called
// before a call's first launch, so the error a failed query leaves can be taken back without
// hiding one of the call's own.
bool capture_of(hipStream_t s, unsigned long long& id) {
    hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
    unsigned long long cid = 0;
    if (hipStreamGetCaptureInfo(s, &st, &cid) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    id = st == hipStreamCaptureStatusActive ? cid : 0ull;
    return true;
}

// Records what a forward call just enqueued left zeroed in `saved` (capture state as queried
// before the call's launches).
void mark_clean(ags_ctx* ctx, const void* saved, unsigned bits, bool known, unsigned long long id) {
    ctx->clean_saved = known ? saved : nullptr;
    ctx->clean_bits = known ? bits : 0u;
    ctx->clean_capture = id;
}

}  // namespace

namespace ags {
StageTimer::StageTimer(ags_ctx* c, int st, hipStream_t str) : ctx(c), stage(st), s(str) {
    if (!ctx->prof) return;
    a = take();
    b = take();
    if (a) (void)hipEventRecord(a, s);
}
hipEvent_t StageTimer::take() {
    if (!ctx->pool.empty()) {
        hipEvent_t e = ctx->pool.back();
        ctx->pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}
StageTimer::~StageTimer() {
    if (!ctx->prof || !a || !b) return;
    (void)hipEventRecord(b, s);
    ctx->pending.push_back({stage, a, b});
}

int ctx_device(const ags_ctx* ctx) { return ctx->device; }
int ctx_record_hip(ags_ctx* ctx, hipError_t e) {
    if (ctx) ctx->last_hip = (int)(e != hipSuccess ? e : hipErrorUnknown);
    return AGS_ERR_HIP;
}
}  // namespace ags

extern "C" {

int ags_version(void) { return AGS_ABI_VERSION; }

const char* ags_error_string(int code) {
    switch (code) {
        case AGS_OK: return "ok";
        case AGS_ERR_INVALID_ARG: return "invalid argument";
        case AGS_ERR_WORKSPACE: return "buffer smaller than required";
        case AGS_ERR_CAPACITY: return "intersection capacity too small";
        case AGS_ERR_HIP: return "HIP runtime error";
        case AGS_ERR_NOT_SUPPORTED: return "not supported";
        default: return "unknown error";
    }
}

int ags_last_hip_error(const ags_ctx* ctx) { return ctx ? ctx->last_hip : 0; }

void ags_config_default(ags_config* c) {
    if (!c) return;
    c->alpha_min = 1.f / 255.f;
    c->alpha_max = 0.99f;
    c->t_min = 1e-4f;
    c->blur = 0.3f;
    c->z_near = 0.2f;
    c->fov_clamp = 1.3f;
    c->bg[0] = c->bg[1] = c->bg[2] = 0.f;
    c->tile = 16;
    c->batch = 256;
    c->px_per_thread = 1;
    c->batch_bwd = 0;
    c->px_per_thread_bwd = 0;
}

int ags_ctx_create(ags_ctx** out, int device, const ags_config* cfg) {
    if (!out) return AGS_ERR_INVALID_ARG;
    *out = nullptr;
    int rc = check_config(cfg);
    if (rc) return rc;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return AGS_ERR_HIP;
    ags_ctx* c = new (std::nothrow) ags_ctx();
    if (!c) return AGS_ERR_HIP;
    c->device = device;
    c->cfg = *cfg;
    c->last_hip = 0;
    c->prof = false;
    rc = lifecycle_static_scratch(device, &c->static_scratch, &c->static_scratch_bytes);
    if (rc) {
        delete c;
        return rc;
    }
    for (int k = 0; k < ST_COUNT; ++k) {
        c->total_ms[k] = 0.0;
        c->launches[k] = 0;
    }
    *out = c;
    return AGS_OK;
}

void ags_ctx_destroy(ags_ctx* ctx) {
    if (!ctx) return;
    for (auto& p : ctx->pending) {
        (void)hipEventDestroy(p.a);
        (void)hipEventDestroy(p.b);
    }
    for (auto e : ctx->pool) (void)hipEventDestroy(e);
    delete ctx;
}

int ags_ctx_set_config(ags_ctx* ctx, const ags_config* cfg) {
    if (!ctx) return AGS_ERR_INVALID_ARG;
    int rc = check_config(cfg);
    if (rc) return rc;
    ctx->cfg = *cfg;
    ctx->clean_saved = nullptr;  // a saved buffer's layout follows the configuration
    return AGS_OK;
}

int ags_buffer_sizes(const ags_config* cfg, const ags_views* views, int32_t n_gaussians,
                     int32_t sh_degree, int64_t isect_capacity, ags_sizes* out) {
    if (!out || sh_degree < 0 || sh_degree > 3) return AGS_ERR_INVALID_ARG;
    int rc = check_config(cfg);
    if (rc) return rc;
    Layout L;
    rc = build_layout(cfg, views, n_gaussians, isect_capacity, L);
    if (rc) return rc;
    out->saved_bytes = L.s_total;
    out->fwd_ws_bytes = L.f_total;
    out->bwd_ws_bytes = L.b_total;
    out->n_pairs = L.Q;
    out->n_pixels = L.P;
    out->n_tiles = L.n_tiles;
    out->tile_bits = L.tile_bits;
    out->off_counters = L.s_counters;
    out->off_records = L.s_records;
    out->off_pair_count = L.s_pair_count;
    out->off_tile_pairs = L.s_tile_pairs;
    out->off_ranges = L.s_ranges;
    out->off_t_final = L.s_t_final;
    out->off_last = L.s_last;
    // keys and values ping-pong together and the values end in `saved` (buffer 0 of the
    // tile sort), so the sorted keys end in the workspace's first key buffer
    out->off_tile_keys = L.f_tkeys0;
    out->off_work = L.s_work;
    out->n_work = raster_blocks(L.vt);
    return AGS_OK;
}

int ags_workspace_query(const ags_ctx* ctx, const ags_views* views, int32_t n_gaussians, int32_t sh_degree,
                        int64_t isect_capacity, ags_sizes* out) {
    if (!ctx) return AGS_ERR_INVALID_ARG;
    return ags_buffer_sizes(&ctx->cfg, views, n_gaussians, sh_degree, isect_capacity, out);
}

int ags_render_fwd(ags_ctx* ctx, const ags_views* views, const ags_gaussians* g,
                   const ags_camera* cams, int64_t isect_capacity, const ags_fwd_out* out,
                   void* saved, void* ws, size_t ws_bytes, void* stream) {
    if (!ctx || !out || !saved || !ws || !cams) return AGS_ERR_INVALID_ARG;
    if (misaligned(saved) || misaligned(ws)) return AGS_ERR_INVALID_ARG;
    int rc = check_gaussians(g);
    if (rc) return rc;
    Layout L;
    rc = build_layout(&ctx->cfg, views, g->n, isect_capacity, L);
    if (rc) return rc;
    if (ws_bytes < L.f_total) return AGS_ERR_WORKSPACE;
    if (L.P > 0 && (!out->rgb || !out->depth || !out->alpha)) return AGS_ERR_INVALID_ARG;
    hipStream_t s = (hipStream_t)stream;
    if (hipSetDevice(ctx->device) != hipSuccess) return hip_status(ctx);
    const Settings st = settings_of(ctx->cfg);
    unsigned long long cid = 0;
    const bool cid_known = capture_of(s, cid);
    ctx->clean_saved = nullptr;
    {
        Scope sc(ctx, ST_PROJECT, s);
        ProjectArgs pa;
        pa.vt = L.vt;
        pa.st = st;
        pa.n = g->n;
        pa.sh_degree = g->sh_degree;
        pa.means = g->means;
        pa.log_scales = g->log_scales;
        pa.quats = g->quats;
        pa.logits = g->opacity_logits;
        pa.sh = g->sh;
        pa.cams = cams;
        pa.records = at<float>(saved, L.s_records);
        pa.pair_count = at<uint32_t>(saved, L.s_pair_count);
        pa.pair_z = at<uint32_t>(ws, L.f_pair_z);
        pa.grad2d = at<float>(saved, L.s_grad2d);
        launch_project_fwd(pa, s);
    }
    {
        Scope sc(ctx, ST_BINNING, s);
        run_binning(bin_args(L, saved, ws), s);
    }
    {
        Scope sc(ctx, ST_RASTER_FWD, s);
        RasterArgs ra;
        ra.vt = L.vt;
        ra.st = st;
        ra.records = at<float>(saved, L.s_records);
        ra.tile_pairs = at<uint32_t>(saved, L.s_tile_pairs);
        ra.ranges = at<uint32_t>(saved, L.s_ranges);
        ra.work = at<uint32_t>(saved, L.s_work);
        ra.rgb = out->rgb;
        ra.depth = out->depth;
        ra.alpha = out->alpha;
        ra.depth_var = out->depth_var;
        ra.t_final = at<float>(saved, L.s_t_final);
        ra.last = at<uint32_t>(saved, L.s_last);
        ra.zero_px[0] = at<float>(saved, L.s_ddepth);
        ra.zero_px[1] = out->depth_var ? at<float>(saved, L.s_ddepth2) : nullptr;
        rc = launch_raster_fwd(ra, ctx->cfg.tile, ctx->cfg.batch, ctx->cfg.px_per_thread, s);
        if (rc) return rc;
    }
    mark_clean(ctx, saved, kClearRows | kClearDepth | (out->depth_var ? kClearDepth2 : 0u), cid_known, cid);
    return hip_status(ctx);
}

int ags_bin_records(ags_ctx* ctx, const ags_views* views, int32_t n_gaussians, const float* records,
                    const uint8_t* valid, int64_t isect_capacity, void* saved, void* ws,
                    size_t ws_bytes, void* stream) {
    if (!ctx || !saved || !ws || (!records && n_gaussians > 0) || (!valid && n_gaussians > 0))
        return AGS_ERR_INVALID_ARG;
    if (misaligned(saved) || misaligned(ws) || misaligned(records)) return AGS_ERR_INVALID_ARG;
    Layout L;
    int rc = build_layout(&ctx->cfg, views, n_gaussians, isect_capacity, L);
    if (rc) return rc;
    if (ws_bytes < L.f_total) return AGS_ERR_WORKSPACE;
    hipStream_t s = (hipStream_t)stream;
    if (hipSetDevice(ctx->device) != hipSuccess) return hip_status(ctx);
    ctx->clean_saved = nullptr;  // the backward of these records clears its accumulators itself
    Scope sc(ctx, ST_BINNING, s);
    if (L.Q > 0)
        (void)hipMemcpyAsync(at<float>(saved, L.s_records), records, (size_t)L.Q * kRecFloats * 4,
                             hipMemcpyDeviceToDevice, s);
    launch_count_from_records(L.vt, records, valid, L.Q, at<uint32_t>(saved, L.s_pair_count),
                              at<uint32_t>(ws, L.f_pair_z), s);
    run_binning(bin_args(L, saved, ws), s);
    return hip_status(ctx);
}

namespace {

// The backward; with `fused` non-null the colour phase of the projection backward also
// applies Adam to every Gaussian parameter (grads->sh is then not written and may be null).
int render_bwd(ags_ctx* ctx, const ags_views* views, const ags_gaussians* g, const ags_camera* cams,
               int64_t isect_capacity, const ags_fwd_out* fwd, void* saved, const ags_upstream* up,
               const ags_loss* loss, ags_grads* grads, float* loss_out, void* ws, size_t ws_bytes, void* stream,
               const AdamArgs* fused) {
    if (!ctx || !saved || !ws || !cams || !grads) return AGS_ERR_INVALID_ARG;
    if (misaligned(saved) || misaligned(ws)) return AGS_ERR_INVALID_ARG;
    if ((up == nullptr) == (loss == nullptr)) return AGS_ERR_INVALID_ARG;
    int rc = check_gaussians(g);
    if (rc) return rc;
    Layout L;
    rc = build_layout(&ctx->cfg, views, g->n, isect_capacity, L);
    if (rc) return rc;
    if (ws_bytes < L.b_total) return AGS_ERR_WORKSPACE;
    if (g->n > 0 && (!grads->means || !grads->log_scales || !grads->quats || !grads->opacity_logits ||
                     (!grads->sh && !fused)))
        return AGS_ERR_INVALID_ARG;
    if (fused && grads->accumulate) return AGS_ERR_INVALID_ARG;
    if (!grads->pose) return AGS_ERR_INVALID_ARG;
    if ((grads->stat_grad == nullptr) != (grads->stat_count == nullptr)) return AGS_ERR_INVALID_ARG;
    long long n_targets = 0;
    if (loss) {
        if (!fwd || !fwd->rgb || !fwd->depth || !loss->gt_rgb) return AGS_ERR_INVALID_ARG;
        if (loss->mask && !loss->l1_count) return AGS_ERR_INVALID_ARG;
        if (!(loss->ssim_weight >= 0.f && loss->ssim_weight <= 1.f)) return AGS_ERR_INVALID_ARG;
        if (loss->sigma_mode != AGS_SIGMA_FIXED && loss->sigma_mode != AGS_SIGMA_RENDERED) return AGS_ERR_INVALID_ARG;
        if (loss->sigma_mode == AGS_SIGMA_RENDERED && (!fwd->depth_var || !(loss->sigma_floor > 0.f)))
            return AGS_ERR_INVALID_ARG;
        if (loss->depth_offsets) {
            if (loss->depth_offsets[0] != 0) return AGS_ERR_INVALID_ARG;
            for (int b = 0; b < views->n_views; ++b)
                if (loss->depth_offsets[b + 1] < loss->depth_offsets[b]) return AGS_ERR_INVALID_ARG;
            n_targets = loss->depth_offsets[views->n_views];
            if (n_targets > 0 && (!loss->depth_pix || !loss->depth_val || !loss->depth_sigma))
                return AGS_ERR_INVALID_ARG;
        }
    }
    hipStream_t s = (hipStream_t)stream;
    if (hipSetDevice(ctx->device) != hipSuccess) return hip_status(ctx);
    const Settings st = settings_of(ctx->cfg);
    float* grad2d = at<float>(saved, L.s_grad2d);
    float* ddepth = at<float>(saved, L.s_ddepth);
    float* ddepth2 = at<float>(saved, L.s_ddepth2);
    const bool rendered_var = loss && loss->sigma_mode == AGS_SIGMA_RENDERED;
    float* partials = at<float>(ws, L.b_partials);
    {
        // the accumulators start at zero: the forward that filled `saved` zeroed them unless
        // another backward (or a call in another capture state) came in between
        unsigned need = kClearRows;
        if (loss && n_targets > 0) need |= kClearDepth;
        if (rendered_var && n_targets > 0) need |= kClearDepth2;
        unsigned long long cid = 0;
        if (ctx->clean_saved == saved && capture_of(s, cid) && cid == ctx->clean_capture) need &= ~ctx->clean_bits;
        ctx->clean_saved = nullptr;  // this backward dirties them
        if (need) {
            Scope sc(ctx, ST_CLEAR, s);
            BwdClearArgs ca;
            memset(&ca, 0, sizeof(ca));
            ca.grad2d = (need & kClearRows) ? grad2d : nullptr;
            ca.pair_count = at<uint32_t>(saved, L.s_pair_count);
            ca.n_pairs = (need & kClearRows) ? L.Q : 0;
            int r = 0;
            if (need & kClearDepth) {
                ca.zero[r] = ddepth;
                ca.zero_n[r++] = L.P;
            }
            if (need & kClearDepth2) {
                ca.zero[r] = ddepth2;
                ca.zero_n[r++] = L.P;
            }
            launch_bwd_clear(ca, s);
        }
    }
    RasterBwdArgs ra;
    memset(&ra, 0, sizeof(ra));
    ra.vt = L.vt;
    ra.st = st;
    ra.records = at<float>(saved, L.s_records);
    ra.tile_pairs = at<uint32_t>(saved, L.s_tile_pairs);
    ra.ranges = at<uint32_t>(saved, L.s_ranges);
    ra.work = at<uint32_t>(saved, L.s_work);
    ra.t_final = at<float>(saved, L.s_t_final);
    ra.last = at<uint32_t>(saved, L.s_last);
    ra.grad2d = grad2d;
    if (loss) {
        ra.loss_mode = 1;
        ra.rgb = fwd->rgb;
        ra.gt_rgb = loss->gt_rgb;
        ra.mask = loss->mask;
        const double ls = loss->ssim_weight > 0.f ? (double)loss->ssim_weight : 0.0;
        SsimArgs sa;
        memset(&sa, 0, sizeof(sa));
        for (int b = 0; b < views->n_views; ++b) {
            const double nb = loss->mask ? (double)loss->l1_count[b]
                                         : (double)views->width[b] * (double)views->height[b];
            ra.l1_scale[b] = nb > 0 ? (float)((1.0 - ls) * loss->w_l1 / (3.0 * nb)) : 0.f;
            sa.scale[b] = nb > 0 ? (float)(ls * loss->w_l1 / (3.0 * nb)) : 0.f;
        }
        if (ls > 0.0) {
            Scope sc(ctx, ST_SSIM, s);
            sa.vt = L.vt;
            sa.rgb = fwd->rgb;
            sa.gt_rgb = loss->gt_rgb;
            sa.mask = loss->mask;
            sa.d_rgb = at<float>(ws, L.b_dssim);
            sa.partials = partials + L.n_tiles + lidar_blocks(0);
            launch_ssim(sa, s);
            ra.d_rgb = sa.d_rgb;
        }
        ra.loss_partials = partials;
        ra.d_depth = n_targets > 0 ? ddepth : nullptr;
        ra.d_depth2 = (n_targets > 0 && rendered_var) ? ddepth2 : nullptr;
        if (n_targets > 0) {
            Scope sc(ctx, ST_LIDAR, s);
            LidarArgs la;
            memset(&la, 0, sizeof(la));
            la.vt = L.vt;
            la.depth = fwd->depth;
            la.depth_var = rendered_var ? fwd->depth_var : nullptr;
            la.sigma_floor = loss->sigma_floor;
            la.d_depth2 = ddepth2;
            la.pix = loss->depth_pix;
            la.val = loss->depth_val;
            la.sigma = loss->depth_sigma;
            la.n_targets = n_targets;
            for (int b = 0; b <= views->n_views; ++b) la.target_off[b] = loss->depth_offsets[b];
            for (int b = 0; b < views->n_views; ++b) {
                const long long nb = loss->depth_offsets[b + 1] - loss->depth_offsets[b];
                la.scale[b] = nb > 0 ? (float)(loss->lambda_lidar / (double)nb) : 0.f;
            }
            la.d_depth = ddepth;
            la.loss_partials = partials + L.n_tiles;  // one slot per LiDAR block
            launch_lidar_adjoint(la, s);
        }
    } else {
        ra.loss_mode = 0;
        ra.d_rgb = up->d_rgb;
        ra.d_depth = up->d_depth;
        ra.d_alpha = up->d_alpha;
    }
    {
        Scope sc(ctx, ST_RASTER_BWD, s);
        const int mb = ctx->cfg.batch_bwd ? ctx->cfg.batch_bwd : ctx->cfg.batch;
        const int pb = ctx->cfg.px_per_thread_bwd ? ctx->cfg.px_per_thread_bwd : ctx->cfg.px_per_thread;
        rc = launch_raster_bwd(ra, ctx->cfg.tile, mb, pb, s);
        if (rc) return rc;
    }
    {
        Scope sc(ctx, ST_PROJECT_BWD, s);
        ProjectBwdArgs pa;
        pa.vt = L.vt;
        pa.st = st;
        pa.n = g->n;
        pa.sh_degree = g->sh_degree;
        pa.means = g->means;
        pa.log_scales = g->log_scales;
        pa.quats = g->quats;
        pa.logits = g->opacity_logits;
        pa.sh = g->sh;
        pa.cams = cams;
        pa.pair_count = at<uint32_t>(saved, L.s_pair_count);
        pa.records = at<float>(saved, L.s_records);
        pa.grad2d = grad2d;
        pa.g_means = grads->means;
        pa.g_log_scales = grads->log_scales;
        pa.g_quats = grads->quats;
        pa.g_logits = grads->opacity_logits;
        pa.g_sh = grads->sh;
        pa.g_pose = grads->pose;
        pa.accumulate = grads->accumulate;
        pa.pose_partials = at<float>(ws, L.b_pose_part);
        pa.vis_mask = at<uint32_t>(ws, L.b_vis);
        pa.stat_grad = grads->stat_grad;
        pa.stat_count = grads->stat_count;
        pa.fused_adam = fused != nullptr;
        if (fused) pa.adam = *fused;
        else memset(&pa.adam, 0, sizeof(pa.adam));
        pa.loss_partials = partials;
        pa.n_loss = L.n_partials;
        pa.loss_skip0 = pa.loss_skip1 = 0;
        pa.loss_out = nullptr;
        if (loss && loss_out) {
            // partials: the tiles', then the LiDAR blocks' and the D-SSIM blocks'; the parts
            // of terms that are off were not written and count as zero
            const long long lidar0 = L.n_tiles, ssim0 = L.n_tiles + lidar_blocks(0);
            const bool no_lidar = n_targets == 0, no_ssim = !(loss->ssim_weight > 0.f);
            pa.loss_skip0 = no_lidar ? lidar0 : (no_ssim ? ssim0 : L.n_partials);
            pa.loss_skip1 = no_ssim ? L.n_partials : (no_lidar ? ssim0 : L.n_partials);
            pa.loss_out = loss_out;
        }
        launch_project_bwd(pa, s);  // its pose reduction also sums the loss partials
    }
    return hip_status(ctx);
}

// Adam arguments from the public structs (validated by the caller).
AdamArgs adam_args(const ags_adam* hp, ags_gaussians* p, const ags_grads* gr, ags_gaussians* m, ags_gaussians* v,
                   const int32_t* step) {
    AdamArgs a;
    memset(&a, 0, sizeof(a));
    a.n = p->n;
    a.sh_k = (p->sh_degree + 1) * (p->sh_degree + 1);
    float* pp[5] = {p->means, p->log_scales, p->quats, p->opacity_logits, p->sh};
    const float* gg[5] = {gr->means, gr->log_scales, gr->quats, gr->opacity_logits, gr->sh};
    float* mm[5] = {m->means, m->log_scales, m->quats, m->opacity_logits, m->sh};
    float* vv[5] = {v->means, v->log_scales, v->quats, v->opacity_logits, v->sh};
    for (int k = 0; k < 5; ++k) {
        a.p[k] = pp[k];
        a.g[k] = gg[k];
        a.m[k] = mm[k];
        a.v[k] = vv[k];
    }
    a.lr[0] = hp->lr_means;
    a.lr[1] = hp->lr_log_scales;
    a.lr[2] = hp->lr_quats;
    a.lr[3] = hp->lr_opacity;
    a.lr[4] = hp->lr_sh0;
    a.lr[5] = hp->lr_shrest;
    a.beta1 = hp->beta1;
    a.beta2 = hp->beta2;
    a.eps = hp->eps;
    a.step = step;
    return a;
}

bool adam_shapes_ok(const ags_gaussians* p, const ags_gaussians* m, const ags_gaussians* v) {
    if (check_gaussians(p) || check_gaussians(m) || check_gaussians(v)) return false;
    return m->n == p->n && v->n == p->n && m->sh_degree == p->sh_degree && v->sh_degree == p->sh_degree;
}

}  // namespace

int ags_render_bwd(ags_ctx* ctx, const ags_views* views, const ags_gaussians* g,
                   const ags_camera* cams, int64_t isect_capacity, const ags_fwd_out* fwd,
                   void* saved, const ags_upstream* up, const ags_loss* loss,
                   ags_grads* grads, float* loss_out, void* ws, size_t ws_bytes, void* stream) {
    return render_bwd(ctx, views, g, cams, isect_capacity, fwd, saved, up, loss, grads, loss_out, ws, ws_bytes,
                      stream, nullptr);
}

int ags_render_bwd_adam(ags_ctx* ctx, const ags_views* views, ags_gaussians* params, const ags_camera* cams,
                        int64_t isect_capacity, const ags_fwd_out* fwd, void* saved,
                        const ags_upstream* up, const ags_loss* loss, ags_grads* grads, float* loss_out,
                        const ags_adam* hp, ags_gaussians* m, ags_gaussians* v, const int32_t* step, void* ws,
                        size_t ws_bytes, void* stream) {
    if (!ctx || !params || !grads || !hp || !m || !v || !step) return AGS_ERR_INVALID_ARG;
    if (!adam_shapes_ok(params, m, v)) return AGS_ERR_INVALID_ARG;
    const AdamArgs a = adam_args(hp, params, grads, m, v, step);
    return render_bwd(ctx, views, params, cams, isect_capacity, fwd, saved, up, loss, grads, loss_out, ws, ws_bytes,
                      stream, &a);
}

int ags_adam_step(ags_ctx* ctx, const ags_adam* hp, ags_gaussians* p, const ags_grads* gr,
                  ags_gaussians* m, ags_gaussians* v, const int32_t* step, void* stream) {
    if (!ctx || !hp || !p || !gr || !m || !v || !step) return AGS_ERR_INVALID_ARG;
    if (!adam_shapes_ok(p, m, v)) return AGS_ERR_INVALID_ARG;
    if (p->n > 0 && (!gr->means || !gr->log_scales || !gr->quats || !gr->opacity_logits || !gr->sh))
        return AGS_ERR_INVALID_ARG;
    hipStream_t s = (hipStream_t)stream;
    if (hipSetDevice(ctx->device) != hipSuccess) return hip_status(ctx);
    const AdamArgs a = adam_args(hp, p, gr, m, v, step);
    Scope sc(ctx, ST_ADAM, s);
    launch_adam(a, s);
    return hip_status(ctx);
}

int ags_lifecycle_workspace(int64_t n, size_t* bytes) {
    if (n < 0 || n > 0x7fffffffLL || !bytes) return AGS_ERR_INVALID_ARG;
    const long long ns = n > 0 ? n : 1;
    *bytes = align_up((size_t)ns * 4) * 2 + align_up((size_t)scan_blocks(ns) * 4);
    return AGS_OK;
}

namespace {

int lifecycle_step(ags_ctx* ctx, const ags_lifecycle* lp, const ags_gaussians* in, const ags_gaussians* in_m,
                   const ags_gaussians* in_v, const float* stat_grad, const float* stat_count,
                   const float* split_noise, ags_gaussians* out, ags_gaussians* out_m, ags_gaussians* out_v,
                   int32_t* n_out_dev, uint8_t* actions_dev, void* ws, size_t ws_bytes, void* stream) {
    if (!ctx || !lp || !in || !in_m || !in_v || !out || !out_m || !out_v || !n_out_dev || !ws)
        return AGS_ERR_INVALID_ARG;
    if (check_gaussians(in) || check_gaussians(in_m) || check_gaussians(in_v) || check_gaussians(out) ||
        check_gaussians(out_m) || check_gaussians(out_v))
        return AGS_ERR_INVALID_ARG;
    const int deg = in->sh_degree;
    if (in_m->n != in->n || in_v->n != in->n || out_m->n != out->n || out_v->n != out->n)
        return AGS_ERR_INVALID_ARG;
    if (in_m->sh_degree != deg || in_v->sh_degree != deg || out->sh_degree != deg || out_m->sh_degree != deg ||
        out_v->sh_degree != deg)
        return AGS_ERR_INVALID_ARG;
    if ((long long)out->n < 2LL * in->n) return AGS_ERR_INVALID_ARG;
    if (lp->do_densify && in->n > 0 && (!stat_grad || !stat_count || !split_noise)) return AGS_ERR_INVALID_ARG;
    if (!(lp->tau_opa >= 0.f && lp->tau_opa < 1.f && lp->s_min >= 0.f && lp->s_max > lp->s_min))
        return AGS_ERR_INVALID_ARG;
    if (lp->do_reset && !(lp->tau_reset > lp->tau_opa && lp->tau_reset < 1.f)) return AGS_ERR_INVALID_ARG;
    if (lp->do_densify && !(lp->split_scale > 0.f)) return AGS_ERR_INVALID_ARG;
    size_t need = 0;
    ags_lifecycle_workspace(in->n, &need);
    if (ws_bytes < need) return AGS_ERR_WORKSPACE;
    hipStream_t s = (hipStream_t)stream;
    if (hipSetDevice(ctx->device) != hipSuccess) return hip_status(ctx);
    LifecycleArgs a;
    memset(&a, 0, sizeof(a));
    a.n = in->n;
    a.k3 = 3 * (deg + 1) * (deg + 1);
    a.cap = out->n;
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
    a.stat_grad = stat_grad;
    a.stat_count = stat_count;
    a.noise = split_noise;
    a.do_prune = lp->do_prune != 0;
    a.do_densify = lp->do_densify != 0;
    a.do_reset = lp->do_reset != 0;
    a.tau_opa = lp->tau_opa;
    a.s_min = lp->s_min;
    a.s_max = lp->s_max;
    a.grad_threshold = lp->grad_threshold;
    a.kappa = lp->kappa;
    a.two_s_init = 2.f * lp->s_init;
    a.tau_reset = lp->tau_reset;
    a.reset_logit = lp->do_reset ? (float)std::log((double)lp->tau_reset / (1.0 - (double)lp->tau_reset)) : 0.f;
    a.log_split = lp->do_densify ? (float)std::log((double)lp->split_scale) : 0.f;
    const long long ns = in->n > 0 ? in->n : 1;
    char* w = static_cast<char*>(ws);
    a.counts = reinterpret_cast<uint32_t*>(w);
    a.offsets = reinterpret_cast<uint32_t*>(w + align_up((size_t)ns * 4));
    a.scan_tmp.block_sums = reinterpret_cast<uint32_t*>(w + 2 * align_up((size_t)ns * 4));
    a.actions = actions_dev;
    a.n_out = n_out_dev;
    Scope sc(ctx, ST_LIFECYCLE, s);
    launch_lifecycle(a, s);
    return hip_status(ctx);
}

}  // namespace

int ags_lifecycle_step(ags_ctx* ctx, const ags_lifecycle* lp, const ags_gaussians* in, const ags_gaussians* in_m,
                       const ags_gaussians* in_v, const float* stat_grad, const float* stat_count,
                       const float* split_noise, ags_gaussians* out, ags_gaussians* out_m, ags_gaussians* out_v,
                       int32_t* n_out_dev, uint8_t* actions_dev, void* ws, size_t ws_bytes, void* stream) {
    return lifecycle_step(ctx, lp, in, in_m, in_v, stat_grad, stat_count, split_noise, out, out_m, out_v, n_out_dev,
                          actions_dev, ws, ws_bytes, stream);
}

int ags_lifecycle_step_noalloc(ags_ctx* ctx, const ags_lifecycle* lp, const ags_gaussians* in,
                               const ags_gaussians* in_m, const ags_gaussians* in_v, const float* stat_grad,
                               const float* stat_count, const float* split_noise, ags_gaussians* out,
                               ags_gaussians* out_m, ags_gaussians* out_v, int32_t* n_out_dev,
                               uint8_t* actions_dev, void* stream) {
    if (!ctx || !in || !ctx->static_scratch) return AGS_ERR_INVALID_ARG;
    if (in->n > AGS_LIFECYCLE_NOALLOC_MAX_N) return AGS_ERR_WORKSPACE;
    // the static array's device address (never the host-side name of the array)
    return lifecycle_step(ctx, lp, in, in_m, in_v, stat_grad, stat_count, split_noise, out, out_m, out_v, n_out_dev,
                          actions_dev, ctx->static_scratch, ctx->static_scratch_bytes, stream);
}

int ags_check_finite(ags_ctx* ctx, const ags_gaussians* g, int32_t* n_bad_dev, void* stream) {
    if (!ctx || !n_bad_dev || check_gaussians(g)) return AGS_ERR_INVALID_ARG;
    hipStream_t s = (hipStream_t)stream;
    if (hipSetDevice(ctx->device) != hipSuccess) return hip_status(ctx);
    launch_fill_u32(reinterpret_cast<uint32_t*>(n_bad_dev), 0u, 1, s);
    const long long n = g->n, k3 = 3LL * (g->sh_degree + 1) * (g->sh_degree + 1);
    launch_count_nonfinite(g->means, 3 * n, n_bad_dev, s);
    launch_count_nonfinite(g->log_scales, 3 * n, n_bad_dev, s);
    launch_count_nonfinite(g->quats, 4 * n, n_bad_dev, s);
    launch_count_nonfinite(g->opacity_logits, n, n_bad_dev, s);
    launch_count_nonfinite(g->sh, k3 * n, n_bad_dev, s);
    return hip_status(ctx);
}

int ags_pose_step(ags_ctx* ctx, const ags_adam* hp, ags_camera* cams, int32_t n_views,
                  const float* pose_grad, float* pose_m, float* pose_v, int32_t* step,
                  int32_t advance_step, void* stream) {
    if (!ctx || !hp || !cams || !pose_grad || !pose_m || !pose_v || !step) return AGS_ERR_INVALID_ARG;
    if (n_views < 1 || n_views > AGS_MAX_VIEWS) return AGS_ERR_INVALID_ARG;
    hipStream_t s = (hipStream_t)stream;
    if (hipSetDevice(ctx->device) != hipSuccess) return hip_status(ctx);
    Scope sc(ctx, ST_POSE, s);
    launch_pose_step(cams, n_views, pose_grad, pose_m, pose_v, step, advance_step, hp->lr_pose, hp->beta1,
                     hp->beta2, hp->eps, s);
    return hip_status(ctx);
}

int ags_profile_enable(ags_ctx* ctx, int enable) {
    if (!ctx) return AGS_ERR_INVALID_ARG;
    ctx->prof = enable != 0;
    return AGS_OK;
}

static int drain(ags_ctx* ctx) {
    for (auto& p : ctx->pending) {
        if (hipEventSynchronize(p.b) != hipSuccess) return hip_status(ctx);
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
            ctx->total_ms[p.stage] += ms;
            ctx->launches[p.stage] += 1;
        }
        ctx->pool.push_back(p.a);
        ctx->pool.push_back(p.b);
    }
    ctx->pending.clear();
    return AGS_OK;
}

int ags_profile_read(ags_ctx* ctx, int n_max, const char** names, double* total_ms, int64_t* launches,
                     int* n_out) {
    if (!ctx || !n_out) return AGS_ERR_INVALID_ARG;
    int rc = drain(ctx);
    if (rc) return rc;
    int n = ST_COUNT < n_max ? ST_COUNT : n_max;
    for (int k = 0; k < n; ++k) {
        if (names) names[k] = kStageNames[k];
        if (total_ms) total_ms[k] = ctx->total_ms[k];
        if (launches) launches[k] = ctx->launches[k];
    }
    *n_out = n;
    return AGS_OK;
}

int ags_profile_reset(ags_ctx* ctx) {
    if (!ctx) return AGS_ERR_INVALID_ARG;
    int rc = drain(ctx);
    for (int k = 0; k < ST_COUNT; ++k) {
        ctx->total_ms[k] = 0.0;
        ctx->launches[k] = 0;
    }
    return rc;
}

extern "C++" {
namespace {

// Device buffers of one tuning trial (freed when the trial set ends).
struct TrialBuffers {
    std::vector<void*> ptrs;
    ~TrialBuffers() { release(); }
    void release() {
        for (void* p : ptrs) (void)hipFree(p);
        ptrs.clear();
    }
    template <typename T>
    T* get(size_t count) {
        void* p = nullptr;
        if (hipMalloc(&p, (count > 0 ? count : 1) * sizeof(T)) != hipSuccess) return nullptr;
        ptrs.push_back(p);
        return static_cast<T*>(p);
    }
};

// Buffers of every trial at one tile size (capacity fixed for that tile size).
struct TileTrial {
    TrialBuffers mem;
    size_t ws_bytes = 0;
    void *saved = nullptr, *fwd_ws = nullptr, *bwd_ws = nullptr;
    ags_fwd_out out{};
    ags_grads gr{};
    float* loss = nullptr;
    int64_t cap = 0;

    int alloc(const Layout& L, const ags_gaussians* g, int n_views) {
        mem.release();
        cap = L.cap;
        saved = mem.get<char>(L.s_total);
        fwd_ws = mem.get<char>(L.f_total);
        bwd_ws = mem.get<char>(L.b_total);
        const size_t P = (size_t)L.P, n = (size_t)g->n, k3 = 3 * (size_t)(g->sh_degree + 1) * (g->sh_degree + 1);
        out.rgb = mem.get<float>(3 * P);
        out.depth = mem.get<float>(P);
        out.alpha = mem.get<float>(P);
        out.depth_var = nullptr;
        gr.means = mem.get<float>(3 * n);
        gr.log_scales = mem.get<float>(3 * n);
        gr.quats = mem.get<float>(4 * n);
        gr.opacity_logits = mem.get<float>(n);
        gr.sh = mem.get<float>(k3 * n);
        gr.pose = mem.get<float>(6 * (size_t)n_views);
        gr.accumulate = 0;
        gr.stat_grad = gr.stat_count = nullptr;
        loss = mem.get<float>(1);
        if (!saved || !fwd_ws || !bwd_ws || !out.rgb || !out.depth || !out.alpha || !gr.means || !gr.log_scales ||
            !gr.quats || !gr.opacity_logits || !gr.sh || !gr.pose || !loss)
            return AGS_ERR_HIP;
        return AGS_OK;
    }
};

}  // namespace
}  // extern "C++"

int ags_tune(ags_ctx* ctx, const ags_views* views, const ags_gaussians* g, const ags_camera* cams,
             const ags_loss* loss, int32_t steps, int32_t warmup, ags_config* best, float* predicted_step_ms,
             ags_tune_entry* report, int32_t n_report_max, int32_t* n_report, void* stream) {
    if (!ctx || !views || !g || !cams || !loss || !best || steps < 1 || warmup < 0) return AGS_ERR_INVALID_ARG;
    if (n_report_max > 0 && !report) return AGS_ERR_INVALID_ARG;
    int rc = check_gaussians(g);
    if (rc) return rc;
    Layout L0;
    rc = build_layout(&ctx->cfg, views, g->n, 0, L0);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    if (hipSetDevice(ctx->device) != hipSuccess) return hip_status(ctx);

    int sh_tile[32], sh_ppt[32], sh_batch[32];
    const int n_shapes = raster_shapes(sh_tile, sh_ppt, sh_batch, 32);
    const ags_config base = ctx->cfg;
    // the caller's profile totals are set aside while the tuner uses the context's timers
    rc = drain(ctx);
    if (rc) return rc;
    const bool prof_was = ctx->prof;
    double saved_ms[ST_COUNT];
    long long saved_launches[ST_COUNT];
    for (int k = 0; k < ST_COUNT; ++k) {
        saved_ms[k] = ctx->total_ms[k];
        saved_launches[k] = ctx->launches[k];
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int n_rep = 0;
    ags_config pick = base;
    double pick_total = 1e300;
    bool found = false;
    rc = AGS_OK;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) rc = AGS_ERR_HIP;
    const int tiles[3] = {8, 16, 32};
    for (int ti = 0; ti < 3 && rc == AGS_OK; ++ti) {
        const int T = tiles[ti];
        int first = -1;
        for (int k = 0; k < n_shapes; ++k)
            if (sh_tile[k] == T) {
                first = k;
                break;
            }
        if (first < 0) continue;
        ags_config cfg = base;
        cfg.tile = T;
        cfg.batch = sh_batch[first];
        cfg.px_per_thread = sh_ppt[first];
        cfg.batch_bwd = cfg.px_per_thread_bwd = 0;
        ctx->cfg = cfg;
        ctx->prof = false;
        // intersection capacity of this tile size: grow until the forward fits, then 15 % headroom
        TileTrial tr;
        int64_t cap = L0.P / 2 > (1 << 16) ? L0.P / 2 : (1 << 16);
        int64_t K = 0;
        for (int attempt = 0; attempt < 4 && rc == AGS_OK; ++attempt) {
            Layout L;
            rc = build_layout(&ctx->cfg, views, g->n, cap, L);
            if (rc) break;
            rc = tr.alloc(L, g, views->n_views);
            if (rc) break;
            rc = ags_render_fwd(ctx, views, g, cams, cap, &tr.out, tr.saved, tr.fwd_ws, L.f_total, stream);
            if (rc) break;
            uint32_t cnt[3] = {0, 0, 0};
            if (hipMemcpyAsync(cnt, at<char>(tr.saved, L.s_counters), sizeof(cnt), hipMemcpyDeviceToHost, s) !=
                    hipSuccess ||
                hipStreamSynchronize(s) != hipSuccess) {
                rc = hip_status(ctx);
                break;
            }
            K = cnt[CNT_K];
            const int64_t want = (int64_t)((double)K * 1.15) + 4096;
            if (!cnt[CNT_OVERFLOW] && cap >= want) break;
            if (want > 0x7fffffffLL) {
                rc = AGS_ERR_CAPACITY;
                break;
            }
            cap = want;
        }
        if (rc) break;
        Layout L;
        rc = build_layout(&ctx->cfg, views, g->n, cap, L);
        if (rc) break;
        double t_first = 0.0, f_first = 0.0, b_first = 0.0;
        double best_f = 1e300, best_b = 1e300;
        int bf = first, bb = first;
        for (int k = 0; k < n_shapes && rc == AGS_OK; ++k) {
            if (sh_tile[k] != T) continue;
            ctx->cfg.batch = sh_batch[k];
            ctx->cfg.px_per_thread = sh_ppt[k];
            ctx->cfg.batch_bwd = ctx->cfg.px_per_thread_bwd = 0;
            ctx->prof = false;
            for (int w = 0; w < warmup && rc == AGS_OK; ++w) {
                rc = ags_render_fwd(ctx, views, g, cams, cap, &tr.out, tr.saved, tr.fwd_ws, L.f_total, stream);
                if (!rc)
                    rc = ags_render_bwd(ctx, views, g, cams, cap, &tr.out, tr.saved, nullptr, loss, &tr.gr, tr.loss,
                                        tr.bwd_ws, L.b_total, stream);
            }
            if (rc) break;
            for (int st = 0; st < ST_COUNT; ++st) {
                ctx->total_ms[st] = 0.0;
                ctx->launches[st] = 0;
            }
            ctx->prof = true;
            if (hipEventRecord(e0, s) != hipSuccess) rc = hip_status(ctx);
            for (int it = 0; it < steps && rc == AGS_OK; ++it) {
                rc = ags_render_fwd(ctx, views, g, cams, cap, &tr.out, tr.saved, tr.fwd_ws, L.f_total, stream);
                if (!rc)
                    rc = ags_render_bwd(ctx, views, g, cams, cap, &tr.out, tr.saved, nullptr, loss, &tr.gr, tr.loss,
                                        tr.bwd_ws, L.b_total, stream);
            }
            if (!rc && (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess))
                rc = hip_status(ctx);
            if (!rc) rc = drain(ctx);
            ctx->prof = false;
            if (rc) break;
            float wall = 0.f;
            (void)hipEventElapsedTime(&wall, e0, e1);
            const double step_ms = wall / steps;
            const double f_ms = ctx->total_ms[ST_RASTER_FWD] / steps;
            const double b_ms = ctx->total_ms[ST_RASTER_BWD] / steps;
            if (n_rep < n_report_max) {
                ags_tune_entry& e = report[n_rep];
                e.tile = T;
                e.batch = sh_batch[k];
                e.px_per_thread = sh_ppt[k];
                e.step_ms = (float)step_ms;
                e.raster_fwd_ms = (float)f_ms;
                e.raster_bwd_ms = (float)b_ms;
                e.intersections = K;
            }
            ++n_rep;
            if (k == first) {
                t_first = step_ms;
                f_first = f_ms;
                b_first = b_ms;
            }
            if (f_ms < best_f) {
                best_f = f_ms;
                bf = k;
            }
            if (b_ms < best_b) {
                best_b = b_ms;
                bb = k;
            }
        }
        if (rc) break;
        // the rest of the first shape's step, plus the fastest forward and backward shapes
        const double total = (t_first - f_first - b_first) + best_f + best_b;
        if (total < pick_total) {
            pick_total = total;
            pick = base;
            pick.tile = T;
            pick.batch = sh_batch[bf];
            pick.px_per_thread = sh_ppt[bf];
            pick.batch_bwd = sh_batch[bb];
            pick.px_per_thread_bwd = sh_ppt[bb];
            found = true;
        }
    }
    // tear down: the caller's profile totals and setting return, the pick is applied; the
    // trial buffers are gone, so no saved buffer counts as zeroed
    ctx->clean_saved = nullptr;
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    for (int k = 0; k < ST_COUNT; ++k) {
        ctx->total_ms[k] = saved_ms[k];
        ctx->launches[k] = saved_launches[k];
    }
    ctx->prof = prof_was;
    if (rc || !found) {
        ctx->cfg = base;
        return rc ? rc : AGS_ERR_NOT_SUPPORTED;
    }
    ctx->cfg = pick;
    *best = pick;
    if (predicted_step_ms) *predicted_step_ms = (float)pick_total;
    if (n_report) *n_report = n_rep;
    return AGS_OK;
}

}  // extern "C"
