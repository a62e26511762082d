/*
 * agsplat -- multi-view differentiable Gaussian-splat rasteriser for MI355X (gfx950).
 *
 * C ABI of libagsplat.so.  Plain pointers and sizes only.  "device" pointers are HIP
 * device memory on the context's GPU; "host" pointers are ordinary process memory.
 *
 * What it computes (AgriGS-SLAM, arXiv 2510.26358):
 *   - Gaussians with mean, covariance from scale and rotation, opacity and SH colour
 *     (Sec. III-B, per-splat parameter equation and Sigma = R S S^T R^T); opacity is the
 *     sigmoid of a trainable logit (Sec. III-B, "Pruning");
 *   - projection to image-space conics Sigma' = J W Sigma W^T J^T (Sec. III-B);
 *   - one shared Gaussian set rendered into B synchronised views in one batch, each
 *     view's gradients updating the same parameters (Sec. III-B, multi-view setting);
 *   - front-to-back alpha compositing of colour, expected depth and alpha per pixel
 *     ("standard 3DGS", Sec. III-B), the expected depth being the mean of the rendered
 *     depth distribution of the LiDAR term (Sec. III-C);
 *   - the loss L1 + lambda_L / |Omega| sum KL(N(D_L, sigma_L^2) || N(mu_u, sigma_u^2))
 *     (Sec. III-C, photometric and probabilistic depth-consistency terms), and its
 *     gradients to every Gaussian parameter and to each camera pose (poses refined by
 *     back-propagating through the projection, Sec. III-C and abstract).
 *
 * Fixed readings where the paper is silent are carried in ags_config (cutoffs, tile
 * size, blur, near plane) and documented there.
 *
 * Conventions common to all calls
 *   - Every function returns 0 (AGS_OK) or a negative AGS_ERR_* code; none aborts or
 *     prints.  After AGS_ERR_HIP, ags_last_hip_error() returns the hipError_t.
 *   - Calls that take `stream` (a hipStream_t; NULL = default stream) only enqueue work:
 *     no allocation, no host synchronisation, so they may be captured into a HIP graph.
 *   - The caller owns every buffer.  The library never keeps a pointer past a call.
 *   - Images of all views live in one flat buffer: view b starts at pixel offset
 *     pix_base[b] = sum_{b'<b} W_b' H_b'; inside a view, pixel (x, y) is y * W + x.
 *     Colour planes are channel-major per view: view b's rgb is [3][H_b][W_b] starting at
 *     element 3 * pix_base[b].
 *   - A "pair" is (view b, Gaussian i) with g_begin[b] <= i < g_end[b]; pairs are numbered
 *     view-major: pair_base[b] + (i - g_begin[b]), pair_base[b] = sum_{b'<b} (g_end - g_begin).
 */
#ifndef AGSPLAT_H
#define AGSPLAT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define AGS_ABI_VERSION 5
#define AGS_MAX_VIEWS 32

enum {
    AGS_OK = 0,
    AGS_ERR_INVALID_ARG = -1,   /* null pointer, bad size/shape, unsupported setting */
    AGS_ERR_WORKSPACE = -2,     /* a buffer is smaller than ags_buffer_sizes requires */
    AGS_ERR_CAPACITY = -3,      /* intersection capacity known on the host to be too small */
    AGS_ERR_HIP = -4,           /* a HIP runtime call failed (see ags_last_hip_error) */
    AGS_ERR_NOT_SUPPORTED = -5  /* valid request the library does not implement */
};

/* Rendering settings.  The paper defers these to "standard 3DGS"; the defaults of
 * ags_config_default() are: alpha_min 1/255 (a Gaussian whose alpha is below it is
 * skipped; the footprint box each Gaussian is binned by is the level of this cutoff),
 * alpha_max 0.99 (alpha clamp), t_min 1e-4 (compositing stops before the
 * transmittance would drop below it; that Gaussian is excluded), blur 0.3 px^2 added to
 * the diagonal of Sigma', z_near 0.2 (Gaussians closer are culled), fov_clamp 1.3 (x/z
 * and y/z clamped to +-1.3 half-FOV tangents inside J only), bg = 0, tile 16, batch 256,
 * one pixel per thread, backward shape = forward shape.  The supported (tile, batch,
 * pixels per thread) launch shapes are (8,64,1) (8,128,1) (16,128,1) (16,256,1) (16,64,2)
 * (16,128,2) (16,256,2) (16,64,4) (32,256,4) (32,512,2); others give AGS_ERR_NOT_SUPPORTED at
 * launch. */
typedef struct ags_config {
    float alpha_min, alpha_max, t_min, blur, z_near, fov_clamp;
    float bg[3];
    int tile;          /* tile edge in pixels: 8, 16 or 32 (binning and raster) */
    int batch;         /* forward: Gaussians staged in LDS per batch: 64, 128, 256 or 512 */
    int px_per_thread; /* forward: pixels per thread: 1, 2 or 4 */
    int batch_bwd;     /* backward launch shape; 0 = same as the forward */
    int px_per_thread_bwd;
} ags_config;

/* Camera b, device array element (64 bytes).  World->camera rotation R (row-major) and
 * translation t: x_cam = R x_world + t.  Pinhole intrinsics; pixel (x, y) has its centre
 * at (x + 0.5, y + 0.5) and a camera point projects to (fx x/z + cx, fy y/z + cy). */
typedef struct ags_camera {
    float R[9];
    float t[3];
    float fx, fy, cx, cy;
} ags_camera;

/* Static shape of a batch of views (host memory).  Must agree with the device cameras. */
typedef struct ags_views {
    int n_views;              /* 1 .. AGS_MAX_VIEWS */
    const int32_t* width;     /* host [n_views], >= 1 */
    const int32_t* height;    /* host [n_views], >= 1 */
    const int32_t* g_begin;   /* host [n_views]: view b sees Gaussians [g_begin, g_end) */
    const int32_t* g_end;     /* host [n_views], 0 <= g_begin <= g_end <= n */
} ags_views;

/* Gaussian parameters, structure-of-arrays, device float32.  K = (sh_degree + 1)^2.
 *   means [3][n], log_scales [3][n] (scale = exp), quats [4][n] (w, x, y, z; any norm),
 *   opacity_logits [n] (opacity = sigmoid), sh [K][3][n] (coefficient k, channel c of
 *   Gaussian i at (k * 3 + c) * n + i; real SH, l-major, m = -l..l, Condon-Shortley phase;
 *   colour = max(0, sum_k Y_k(d) sh_k + 0.5), d the unit direction camera centre -> mean).
 * Arithmetic is float32 except the world -> camera transform R mu + t and the camera-centre
 * offset mu + R^T t, which are evaluated in float64 and rounded once, so Gaussians and
 * cameras far from the frame origin (one global map, kilometres across) project as the
 * float32 inputs define, without the cancellation a float32 transform would suffer. */
typedef struct ags_gaussians {
    int32_t n;
    int32_t sh_degree;        /* 0 .. 3 */
    float* means;
    float* log_scales;
    float* quats;
    float* opacity_logits;
    float* sh;
} ags_gaussians;

/* Gradients, same layouts as ags_gaussians, plus pose [n_views][6] = dL/d delta_b for the
 * left perturbation W_b <- Exp(delta_b) W_b, delta = (rho, phi), translation first.
 * accumulate = 0 overwrites every element; 1 adds to what is there. */
typedef struct ags_grads {
    float* means;
    float* log_scales;
    float* quats;
    float* opacity_logits;
    float* sh;
    float* pose;
    int32_t accumulate;
    /* Densification statistic (Sec. III-B lifecycle), each [n] or NULL: for every view in
     * which Gaussian i's footprint rectangle meets the image, stat_grad[i] += |dL/d(u, v)|
     * (the loss gradient at the projected centre, pixel units) and stat_count[i] += 1.
     * Always accumulated (never overwritten); the caller zeroes them after densifying. */
    float* stat_grad;
    float* stat_count;
} ags_grads;

/* Forward outputs (device float32): rgb [3 * P], depth [P] (expected depth: sum of
 * w_i z_i, unnormalised, z the camera-frame depth of the mean), alpha [P] (the accumulated
 * sum of w_i, written as 1 - the final transmittance); P = total pixels. */
typedef struct ags_fwd_out {
    float* rgb;
    float* depth;
    float* alpha;
    float* depth_var; /* [P] or NULL: variance of the rendered depth distribution,
                         sum_k w_k z_k^2 - (sum_k w_k z_k)^2 (needed by the rendered-variance
                         LiDAR term), written when non-null; accumulated as the scatter about
                         the running weighted mean plus A T m^2 (A = sum w, T = final
                         transmittance, m = mean), which avoids the cancellation of the
                         difference of moments in float32 */
} ags_fwd_out;

/* Upstream gradients dL/d(rgb, depth, alpha) in the output layouts; each may be NULL (0). */
typedef struct ags_upstream {
    const float* d_rgb;
    const float* d_depth;
    const float* d_alpha;
} ags_upstream;

/* Fused loss (Sec. III-C: photometric L_3DGS plus L_LiDAR), summed over views b:
 *   w_l1 [(1 - ssim_weight) / (3 n_b) sum_{p in mask_b} sum_c |rgb - gt_rgb|
 *         + ssim_weight / (3 n_b) sum_{p in mask_b} sum_c (1 - ssim_c(p))]
 * + lambda_lidar / |Omega_b| sum_{j in Omega_b} KL(N(D_j, s_j^2) || N(depth(p_j), su_j^2))
 * with su_j = s_j (AGS_SIGMA_FIXED; the KL is then (depth - D_j)^2 / (2 s_j^2)) or
 * su_j^2 = depth_var(p_j) + sigma_floor (AGS_SIGMA_RENDERED: the variance of the rendered
 * depth distribution; the backward then needs fwd->depth_var).  n_b = l1_count[b] if mask is given,
 * else W_b H_b; the sign of 0 is 0.  Repeated target pixels simply add their terms.
 * ssim_c(p) uses the whole rendered view (zero outside it), also outside the mask. */
enum { AGS_SIGMA_FIXED = 0, AGS_SIGMA_RENDERED = 1 };

typedef struct ags_loss {
    const float* gt_rgb;          /* device, rgb layout */
    const uint8_t* mask;          /* device [P] (1 = pixel enters the L1 term) or NULL */
    const int64_t* l1_count;      /* host [n_views]; required when mask != NULL */
    const int32_t* depth_pix;     /* device [n_targets]: pixel index y * W + x in its view, in
                                     [0, W_b H_b).  The call cannot read device data to refuse a
                                     target outside its view: such a target gets no adjoint and
                                     makes the loss (loss_out) NaN, so it cannot pass unnoticed */
    const float* depth_val;       /* device [n_targets]: LiDAR depth D_j (camera z) */
    const float* depth_sigma;     /* device [n_targets]: s_j > 0 */
    const int64_t* depth_offsets; /* host [n_views + 1]: targets of view b are
                                     [depth_offsets[b], depth_offsets[b+1]) */
    float w_l1;
    float lambda_lidar;
    int32_t sigma_mode;           /* AGS_SIGMA_FIXED or AGS_SIGMA_RENDERED */
    float sigma_floor;            /* m^2 added to the rendered variance (> 0 in RENDERED mode) */
    float ssim_weight;            /* lambda of L_3DGS = (1 - lambda) L1 + lambda D-SSIM (Sec. III-C),
                                     in [0, 1]; 0 = L1 only.  D-SSIM = 1 - SSIM with an 11 x 11
                                     Gaussian window (sigma 1.5, zero padding), C1 = 0.01^2,
                                     C2 = 0.03^2, per channel, averaged over the same pixels as
                                     the L1 term (the whole view, or the mask); both parts carry
                                     w_l1. */
} ags_loss;

/* Buffer sizes and the layout of the `saved` buffer (byte offsets), for a batch shape. */
typedef struct ags_sizes {
    size_t saved_bytes;      /* state the forward leaves for the backward, including the
                                backward's accumulators (per-pair 2D adjoint rows, dense
                                depth adjoints), which the forward leaves zeroed */
    size_t fwd_ws_bytes;     /* forward scratch */
    size_t bwd_ws_bytes;     /* backward scratch */
    int64_t n_pairs, n_pixels, n_tiles;
    int32_t tile_bits;       /* bits of the global tile id */
    /* offsets into `saved` */
    size_t off_counters;     /* uint32[5]: K (all candidate intersections), V (visible
                                pairs), overflow flag (K > capacity), K kept (min(K,
                                capacity)), L (intersections in the tile lists: the kept
                                candidates whose tile the alpha >= alpha_min ellipse reaches) */
    size_t off_records;      /* float[n_pairs][12]: u, v, conic a, b, c, opacity, z,
                                ex, ey, r, g, b (written only for visible pairs) */
    size_t off_pair_count;   /* uint32[n_pairs]: tiles touched (0 = culled / off-screen) */
    size_t off_tile_pairs;   /* uint32[capacity]: the first L entries are pair ids, grouped
                                by global tile and ordered by (float32 depth bits, pair id)
                                inside a tile */
    size_t off_ranges;       /* uint32[n_tiles][2]: [start, end) into tile_pairs */
    size_t off_t_final;      /* float[P]: final transmittance */
    size_t off_last;         /* uint32[P]: tile-list entries up to the last contributor */
    size_t off_tile_keys;    /* (forward workspace) uint32[capacity]: sorted global tile ids */
    size_t off_work;         /* uint32[n_work]: the tile of each raster workgroup (see below) */
    int64_t n_work;          /* raster workgroups: strips of 8 tiles go round-robin to eight
                                lists (workgroup g in list g mod 8), each list holds its tiles
                                by descending list length (4 log2(length + 1) buckets) and is
                                padded to equal length with 0xFFFFFFFF (no tile) */
} ags_sizes;

typedef struct ags_ctx ags_ctx;

int ags_version(void);
const char* ags_error_string(int code);
int ags_last_hip_error(const ags_ctx* ctx);
void ags_config_default(ags_config* cfg);

/* Create a context on HIP device `device` with a copy of *cfg.  One context per stream
 * at a time (the context holds timing events).  Errors: INVALID_ARG (bad cfg), HIP. */
int ags_ctx_create(ags_ctx** out, int device, const ags_config* cfg);
void ags_ctx_destroy(ags_ctx* ctx);
int ags_ctx_set_config(ags_ctx* ctx, const ags_config* cfg);

/* Host-only arithmetic: sizes of the buffers fwd/bwd need for this shape and capacity
 * (maximum number of (tile, Gaussian) intersections).  No device access.  The `saved` and
 * `ws` buffers passed to ags_render_fwd / ags_render_bwd / ags_bin_records (and the records
 * of ags_bin_records) must start on a 16-byte boundary, as hipMalloc'd and torch-allocated
 * memory does; otherwise those calls return AGS_ERR_INVALID_ARG. */
int ags_buffer_sizes(const ags_config* cfg, const ags_views* views, int32_t n_gaussians,
                     int32_t sh_degree, int64_t isect_capacity, ags_sizes* out);

/* The same query keyed on a context (its configuration): the workspace sizes of
 * ags_render_fwd / ags_render_bwd for this batch shape under the context's tile size. */
int ags_workspace_query(const ags_ctx* ctx, const ags_views* views, int32_t n_gaussians, int32_t sh_degree,
                        int64_t isect_capacity, ags_sizes* out);

/* Forward render of all views in one batch (Sec. III-B: the splats projected through each
 * camera, Sigma' = J W Sigma W^T J^T, its 2 x 2 block rendered; the B synchronised views of
 * the multi-view setting rendered together, the batch rasterisation of the abstract; colour,
 * expected depth (the mean of the rendered depth distribution of Sec. III-C) and alpha
 * composited front to back): projection, binning, depth/tile sort, tile ranges,
 * compositing.  cams: device [n_views].  saved: device, saved_bytes; ws: device,
 * fwd_ws_bytes.  If the intersections exceed isect_capacity the overflow counter in
 * `saved` is set and the outputs are not valid: enlarge the capacity and run again.  Errors:
 * INVALID_ARG (null or misaligned buffers, bad shapes), WORKSPACE (ws_bytes too small),
 * NOT_SUPPORTED (a launch shape not compiled), HIP. */
int ags_render_fwd(ags_ctx* ctx, const ags_views* views, const ags_gaussians* g,
                   const ags_camera* cams, int64_t isect_capacity, const ags_fwd_out* out,
                   void* saved, void* ws, size_t ws_bytes, void* stream);

/* Backward (Sec. III-C: the multimodal loss back-propagated to every splat parameter and,
 * through the projection model, to each camera pose; the views' gradients summed into the one
 * shared splat set of Sec. III-B).  Exactly one of `up` (upstream gradients) or `loss` (fused
 * loss; then `loss_out`, device float[1] or NULL, receives the loss value) is non-NULL.
 * `fwd` holds the outputs of the matching forward (read in loss mode).  saved: from that
 * forward (transmittance is recomputed from it, no per-pixel blend lists are kept); the
 * backward accumulates into the adjoint buffers it holds, which that forward left zeroed.
 * When the call directly follows, on this context and in the same stream-capture state (both
 * outside any capture, or in one capture), the forward that filled `saved`, it relies on that
 * zeroing; otherwise (a second backward of one forward, say) it clears them first.  (So a captured graph holding a backward but not its forward must not be replayed
 * twice after one forward.)  ws: device, bwd_ws_bytes.  Gradients per ags_grads.  Errors:
 * INVALID_ARG, WORKSPACE, NOT_SUPPORTED, HIP. */
int ags_render_bwd(ags_ctx* ctx, const ags_views* views, const ags_gaussians* g,
                   const ags_camera* cams, int64_t isect_capacity, const ags_fwd_out* fwd,
                   void* saved, const ags_upstream* up, const ags_loss* loss,
                   ags_grads* grads, float* loss_out, void* ws, size_t ws_bytes, void* stream);

/* Binning stage alone (for tests and tuning): from projected records (float[n_pairs][12],
 * the `saved` record layout) and per-pair validity (uint8[n_pairs]), compute pair tile
 * counts, the depth-ordered per-tile pair lists and the ranges into `saved`. */
int ags_bin_records(ags_ctx* ctx, const ags_views* views, int32_t n_gaussians,
                    const float* records, const uint8_t* valid, int64_t isect_capacity,
                    void* saved, void* ws, size_t ws_bytes, void* stream);

/* Adam on the Gaussian parameters (in place).  lr per group: means, log_scales, quats,
 * opacity_logits, sh degree 0, sh degree >= 1.  m, v: device state in the parameter
 * layouts (zero before the first step).  step: device int32, the 1-based step number. */
typedef struct ags_adam {
    float lr_means, lr_log_scales, lr_quats, lr_opacity, lr_sh0, lr_shrest, lr_pose;
    float beta1, beta2, eps;
} ags_adam;

int ags_adam_step(ags_ctx* ctx, const ags_adam* hp, ags_gaussians* params,
                  const ags_grads* grads, ags_gaussians* m, ags_gaussians* v,
                  const int32_t* step, void* stream);

/* The backward of ags_render_bwd followed by ags_adam_step on `params`, in one pass over
 * the Gaussians: the kernel that completes each Gaussian's gradient (the colour adjoint
 * through the SH evaluation, Sec. III-C, joined with the geometry part) applies Adam to all of
 * its parameters in place, so the SH gradient, 48 of a degree-3 Gaussian's 59 values, is
 * never written to or re-read from memory.  Arguments as for ags_render_bwd and
 * ags_adam_step; `grads` still receives the pose gradient, the densification statistic if
 * requested and the geometry gradients (means without the SH direction term, log_scales,
 * quats, opacity_logits), while grads->sh is not written and may be NULL; grads->accumulate
 * must be 0.  The result equals the two calls in sequence. */
int ags_render_bwd_adam(ags_ctx* ctx, const ags_views* views, ags_gaussians* params,
                        const ags_camera* cams, int64_t isect_capacity, const ags_fwd_out* fwd,
                        void* saved, const ags_upstream* up, const ags_loss* loss,
                        ags_grads* grads, float* loss_out, const ags_adam* hp, ags_gaussians* m,
                        ags_gaussians* v, const int32_t* step, void* ws, size_t ws_bytes,
                        void* stream);

/* Adam on each view's se(3) increment (pose_m, pose_v: device float[n_views][6]), then
 * the left retraction W_b <- Exp(delta_b) W_b written into cams; if advance_step != 0 the
 * device step counter is incremented afterwards (end of an optimisation step). */
int ags_pose_step(ags_ctx* ctx, const ags_adam* hp, ags_camera* cams, int32_t n_views,
                  const float* pose_grad, float* pose_m, float* pose_v, int32_t* step,
                  int32_t advance_step, void* stream);

/* Autotuner for the raster launch shapes (tiling is "standard 3DGS" in Sec. III-B; the paper
 * names no tile size or batch).  For every tile size in {8, 16, 32} and every (LDS batch,
 * pixels per thread) shape compiled for it (the list under ags_config), times `steps`
 * forward + fused-loss backward steps of this workload (views, g, cams, loss as for
 * ags_render_fwd / ags_render_bwd), after `warmup` untimed ones, on `stream` with HIP events
 * per stage.  Per tile size it takes the forward shape with the fastest raster forward and
 * the backward shape with the fastest raster backward, predicts the step as the rest of the
 * first shape's step plus those two, and picks the tile size with the fastest prediction.
 * The pick (other fields from the context's configuration) is written to *best and set on
 * the context; *predicted_step_ms (nullable) receives its predicted step time.  report
 * (nullable unless n_report_max > 0) receives up to n_report_max per-shape timings and
 * *n_report (nullable) the number of shapes timed.  Off the hot path: it allocates its trial
 * buffers (device memory for outputs, gradients and the saved state at each tile size's
 * intersection capacity, freed before it returns) and synchronises with the host; g is only
 * read.  The caller's profile totals are kept.  Errors: INVALID_ARG, CAPACITY (more than
 * 2^31 intersections), HIP (allocation or launch; the context keeps its configuration). */
typedef struct ags_tune_entry {
    int32_t tile, batch, px_per_thread;
    float step_ms, raster_fwd_ms, raster_bwd_ms;
    int64_t intersections;  /* K at this tile size */
} ags_tune_entry;

int ags_tune(ags_ctx* ctx, const ags_views* views, const ags_gaussians* g, const ags_camera* cams,
             const ags_loss* loss, int32_t steps, int32_t warmup, ags_config* best, float* predicted_step_ms,
             ags_tune_entry* report, int32_t n_report_max, int32_t* n_report, void* stream);

/* Debug aid, off the hot path: the number of non-finite values (NaN, +-inf) among all of
 * g's parameters, written to *n_bad_dev (device int32).  Enqueued on the stream, no host
 * synchronisation. */
int ags_check_finite(ags_ctx* ctx, const ags_gaussians* g, int32_t* n_bad_dev, void* stream);

/* Per-stage GPU time of the calls since the last reset (HIP events on the calls' streams;
 * enabling adds an event pair per kernel launch).  names: host array of n_max C strings. */
int ags_profile_enable(ags_ctx* ctx, int enable);
int ags_profile_read(ags_ctx* ctx, int n_max, const char** names, double* total_ms,
                     int64_t* launches, int* n_out);
int ags_profile_reset(ags_ctx* ctx);

/* Gaussian-splat lifecycle operations (Sec. III-B "Gaussian Splats Lifecycle Operations"):
 * pruning, gradient-driven densification and opacity reset.  With s_i = exp(max log-scale)
 * (largest axis), o_i = sigmoid(logit), g_i = stat_grad[i] / max(stat_count[i], 1):
 *   prune (do_prune)    if o_i < tau_opa or s_i > s_max or s_i < s_min;
 *   split (do_densify)  else if stat_count[i] > 0, g_i > grad_threshold and s_i > kappa: two
 *                       children at mu + R(q) diag(s) eps_k (eps = split_noise[i][k][0..2],
 *                       standard normals supplied by the caller), log-scales minus
 *                       ln(split_scale), quaternion / opacity / SH copied;
 *   duplicate           else if that gradient test holds and s_i <= 2 s_init: the original and
 *                       an exact copy;
 *   opacity reset (do_reset) if not pruned, tau_opa <= o_i < tau_reset and s_min < s_i < s_max:
 *                       the logit of every output of i becomes logit(tau_reset).
 * Decisions are taken in float32.  Outputs keep input order (a Gaussian's outputs are
 * consecutive); the Adam moments of copies and children are 0, survivors keep theirs. */
typedef struct ags_lifecycle {
    int32_t do_prune, do_densify, do_reset;
    float tau_opa;          /* 0.01 (the paper's value) */
    float s_min, s_max;     /* 5e-5, 0.3 (the paper's values) */
    float grad_threshold;   /* gamma_g, pixel units */
    float kappa;            /* split above this size */
    float s_init;           /* duplicate at or below 2 s_init */
    float tau_reset;        /* reset band upper bound and reset value, in (tau_opa, 1) */
    float split_scale;      /* 1.6 */
} ags_lifecycle;

/* Scratch bytes ags_lifecycle_step needs for n Gaussians. */
int ags_lifecycle_workspace(int64_t n, size_t* bytes);

/* One lifecycle pass over `in` (+ its Adam moments in_m, in_v, same layout), writing to
 * `out` / `out_m` / `out_v` (distinct buffers, same sh_degree, room for out_capacity >= 2 n
 * Gaussians: their `n` fields give the capacity).  stat_grad / stat_count: the statistic
 * above, device float[n] each; split_noise: device float[n][2][3]; all three are required
 * when do_densify != 0 and n > 0, and ignored otherwise.  Writes the new count to *n_out_dev
 * (device int32) and, if non-null, the action of each input to actions_dev[n] (0 keep,
 * 1 prune, 2 duplicate, 3 split).  No host sync, no
 * allocation.  INVALID_ARG for bad pointers, sizes or thresholds, WORKSPACE_TOO_SMALL. */
int ags_lifecycle_step(ags_ctx* ctx, const ags_lifecycle* lp, const ags_gaussians* in,
                       const ags_gaussians* in_m, const ags_gaussians* in_v, const float* stat_grad,
                       const float* stat_count, const float* split_noise, ags_gaussians* out,
                       ags_gaussians* out_m, ags_gaussians* out_v, int32_t* n_out_dev,
                       uint8_t* actions_dev, void* ws, size_t ws_bytes, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): ags_lifecycle_step with its scratch
 * (per-Gaussian output counts, first output slots and scan block sums) in a static device
 * array of the library instead of the `ws` argument.  That array is AGS_LIFECYCLE_NOALLOC_BYTES
 * (32 MiB + 64 KiB) on every GPU the library runs on, held until the process ends; its
 * address is looked up in ags_ctx_create.  Allocates nothing and does not synchronise.
 * in->n must be <= AGS_LIFECYCLE_NOALLOC_MAX_N (2^22) or the call returns
 * AGS_ERR_WORKSPACE; other arguments and errors as ags_lifecycle_step, with the same results.
 * All calls on one GPU share the array and nothing in it needs clearing (every call writes
 * what it reads): calls that can overlap on one GPU (several streams or host threads) race
 * and must be serialised by the caller. */
#define AGS_LIFECYCLE_NOALLOC_MAX_N (1 << 22)
#define AGS_LIFECYCLE_NOALLOC_BYTES ((32u << 20) + (64u << 10))
int ags_lifecycle_step_noalloc(ags_ctx* ctx, const ags_lifecycle* lp, const ags_gaussians* in,
                               const ags_gaussians* in_m, const ags_gaussians* in_v, const float* stat_grad,
                               const float* stat_count, const float* split_noise, ags_gaussians* out,
                               ags_gaussians* out_m, ags_gaussians* out_v, int32_t* n_out_dev,
                               uint8_t* actions_dev, void* stream);

/* ---- Voxel-hashed Gaussian map with a bounded GPU-resident set (Sec. III-B "Incremental
 * Gaussian Mapping": the voxel key equation; "Memory Management": least-recently-used
 * offload to host memory above a threshold tau, reload when a key is met again; with
 * "Gaussian Splats Lifecycle Operations" for pruned and densified splats).
 *
 * Key of a point p: c = floor(p / v) per axis (float32 division and floor), k = (c_x P1 +
 * c_y P2 + c_z P3) mod 2^64 (two voxels whose keys collide are merged); the key 2^64 - 1 is
 * reserved and becomes 2^64 - 2.  |p / v| must stay below 2^62.  A key names a group of
 * splats: the one its first point made and that splat's descendants by densification
 * (ags_map_lifecycle: a copy or split child inherits its parent's key and last_used); keys
 * are not recomputed as means move.  Each splat has an id (never reused) in one of three
 * states: resident (a row of the resident set, the rows the caller renders and optimises),
 * offloaded (its row in the host store) or retired (pruned).  A key whose group has no live
 * member is absent from the map.
 * An insertion call takes its points in order: a key present marks every live member of its
 * group used; an absent key makes one splat from the first point carrying it (mean p,
 * log-scales ln s_init, identity quaternion, logit of o_init, SH DC (rgb - 1/2) / Y_0^0,
 * other SH and Adam moments 0), ids counting up in that order.  A point's id is its group's
 * smallest live id.  Every live splat in a group hit by call t gets last_used = t.  The
 * resident set is rebuilt as: the input rows in order, then the call's new splats (id order),
 * then the members of the groups it hit that were offloaded (reloaded from the host store, id
 * order); while more than tau rows remain, the least recently used (smallest last_used, ties:
 * earlier row) are offloaded to the host store with their current values, the others keeping
 * their order. */
typedef struct ags_map ags_map;

typedef struct ags_map_config {
    float voxel;           /* v, metres, > 0 */
    float s_init;          /* new splat: scale (all axes), > 0 */
    float o_init;          /* new splat: opacity, in (0, 1) */
    int32_t sh_degree;     /* 0..3 */
    uint64_t prime[3];     /* P1, P2, P3 */
    int64_t max_ids;       /* splats the map can ever hold, <= 2^30 */
    int64_t max_points;    /* points per insertion call, <= 2^28 */
    int64_t tau;           /* resident-set bound, >= 1 */
} ags_map_config;

typedef struct ags_map_counts {
    int64_t n_ids;         /* ids handed out so far (all states) */
    int64_t n_resident;    /* rows of the output resident set */
    int64_t n_new, n_reloaded, n_evicted;  /* by this call (n_new: new ids) */
    int64_t n_offloaded;   /* ids in the host store after the call */
    int64_t n_retired;     /* ids this call retired */
} ags_map_counts;

/* voxel 0.05, s_init 0.005, o_init 0.1, degree 3, primes 73856093, 19349663, 83492791,
 * max_ids 2^22, max_points 2^20, tau 2^20. */
int ags_map_config_default(ags_map_config* cfg);

/* Allocates the map on ctx's device: the hash table (open addressing, 2^ceil(log2(2 max_ids))
 * slots of 16 B), per-id key / last_used / residency (13 B), per-point and per-row scratch,
 * device and pinned host staging of max_points rows, and the host store (max_ids rows of
 * 3 x 4 x (11 + 3 (deg+1)^2) bytes, committed as rows are offloaded).  destroy frees it all. */
int ags_map_create(ags_ctx* ctx, const ags_map_config* cfg, ags_map** out);
int ags_map_destroy(ags_map* map);

/* One insertion call (number `frame`, non-decreasing over calls, >= 0).  points / colors:
 * device float[n_points][3] (xyz; rgb in [0, 1]).  in / in_m / in_v / in_ids: the resident set
 * this map returned last (by ags_map_insert or ags_map_lifecycle; values may have changed,
 * not rows or order; n = 0 before the first call); in->n must equal that set's size and every
 * id must be resident and appear once (checked on the device first: INVALID_ARG, nothing
 * changed).  out / out_m / out_v / out_ids: other buffers receiving the new resident set,
 * packed with row stride counts->n_resident; their `n` gives the capacity in rows, which
 * must be >= min(in->n + n_points + n_offloaded, tau) (n_offloaded as the previous call
 * reported it).  point_id: device int32[n_points] (or NULL): the id of each point.
 * evicted_ids: device int32 (or NULL) with room for max(n_points, in->n + n_points +
 * n_offloaded - tau) entries (n_points suffices while ags_map_lifecycle is not used): the ids
 * offloaded by this call, in row order.  Host-synchronous: returns after the stream's work
 * (three synchronisations: the ids check, the reload list, then the new resident set).  The
 * offloaded rows leave for pinned memory on a copy stream of the map's own, which waits for
 * them to be staged and then overlaps whatever the caller enqueues next; a host thread waits
 * for that copy and writes the rows into the host store, and the next call on the map waits
 * for it first (so do ags_map_sync, ags_map_read_store and ags_map_destroy; a failed copy
 * makes the next of them return AGS_ERR_HIP).  When more than max_points rows are reloaded or
 * offloaded, the rows go through the staging in chunks of max_points on the calling thread
 * and are in the host store when the call returns.  INVALID_ARG for bad pointers, sizes or
 * ids, CAPACITY when n_ids + n_points > max_ids (nothing changed); after AGS_ERR_HIP the
 * map's state is undefined (destroy it). */
int ags_map_insert(ags_map* map, const float* points, const float* colors, int64_t n_points, int32_t frame,
                   const ags_gaussians* in, const ags_gaussians* in_m, const ags_gaussians* in_v,
                   const int32_t* in_ids, ags_gaussians* out, ags_gaussians* out_m, ags_gaussians* out_v,
                   int32_t* out_ids, int32_t* point_id, int32_t* evicted_ids, ags_map_counts* counts,
                   void* stream);

/* The map's side of a lifecycle pass (Sec. III-B "Gaussian Splats Lifecycle Operations" over
 * the splats of "Incremental Gaussian Mapping") run on the resident set this map returned
 * last: ids: device int32[n], that set's ids in row order (n = its size); actions: device
 * uint8[n], the pass's action per row as ags_lifecycle_step writes them (0 keep, 1 prune,
 * 2 duplicate, 3 split).  The pass's output rows, in its order, become the resident set:
 * each input's first output keeps the input's id; the second output of a duplicated or split
 * input gets a new id (counting up from n_ids in input order) with the input's key and
 * last_used; a pruned input's id is retired, and a key whose group loses its last live member
 * leaves the map.  rows / rows_m / rows_v: the pass's output rows and moments as
 * ags_lifecycle_step wrote them (row stride = their `n`, its output capacity).  out / out_m /
 * out_v / out_ids: other buffers receiving the new resident set, packed with row stride
 * counts->n_resident (capacity in their `n`, >= that count; out_ids: device int32 with room for
 * 2 n entries).  The resident set may now exceed tau; the next insertion call offloads the
 * excess.  Host-synchronous (two synchronisations).  INVALID_ARG: bad pointers or sizes, n
 * differs from the resident set's size, an id is not resident or appears twice, an action is
 * above 3, or the rows' stride or the output capacity is below the output count (nothing
 * changed); CAPACITY: n_ids + (new ids) > max_ids (nothing changed). */
int ags_map_lifecycle(ags_map* map, const int32_t* ids, const uint8_t* actions, int64_t n,
                      const ags_gaussians* rows, const ags_gaussians* rows_m, const ags_gaussians* rows_v,
                      ags_gaussians* out, ags_gaussians* out_m, ags_gaussians* out_v, int32_t* out_ids,
                      ags_map_counts* counts, void* stream);

/* Waits until the host store holds the rows the last call offloaded; AGS_ERR_HIP if their
 * copy failed. */
int ags_map_sync(ags_map* map);

/* Copies per-id state to host memory (any pointer may be NULL): keys[n_ids], last_used[n_ids],
 * resident[n_ids] (state: 0 offloaded, 1 resident, 2 retired); and, for table_slots (>= the
 * table's slot count, reported in *n_slots), the table's keys and values (a slot keeps a key
 * once entered; its value is the group's smallest live id, -1 while the group is empty; an
 * empty slot: key 2^64 - 1, value -1).  Synchronous. */
int ags_map_export(ags_map* map, uint64_t* keys, int32_t* last_used, uint8_t* resident, uint64_t* table_keys,
                   int32_t* table_ids, int64_t table_slots, int64_t* n_ids, int64_t* n_slots);

/* Rows of offloaded ids from the host store into host memory rows[n][3 F] (F = 11 + 3 (deg+1)^2:
 * parameters, then Adam m, then v; each as means 3, log-scales 3, quaternion 4, logit 1,
 * SH (deg+1)^2 x 3).  INVALID_ARG if an id is out of range, resident or retired. */
int ags_map_read_store(ags_map* map, const int32_t* ids, int64_t n, float* rows);

#ifdef __cplusplus
}
#endif
#endif /* AGSPLAT_H */
