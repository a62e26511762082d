"""ctypes view of libagsplat.so (the C ABI declared in include/agsplat.h).

Argument marshalling only: structures mirror the header field by field.  Loading fails
loudly when the library has not been built -- there is no fallback implementation.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
# AGS_LIBRARY selects another build of the same library (the host-sanitized one, for its test)
LIB_PATH = os.environ.get("AGS_LIBRARY") or os.path.join(HERE, "libagsplat.so")

AGS_OK = 0
AGS_ERR_INVALID_ARG = -1
AGS_ERR_WORKSPACE = -2
AGS_ERR_CAPACITY = -3
AGS_ERR_HIP = -4
AGS_ERR_NOT_SUPPORTED = -5
AGS_MAX_VIEWS = 32
LIFECYCLE_NOALLOC_MAX_N = 1 << 22

EXPORTED = [
    "ags_version", "ags_error_string", "ags_last_hip_error", "ags_config_default",
    "ags_ctx_create", "ags_ctx_destroy", "ags_ctx_set_config", "ags_buffer_sizes", "ags_workspace_query",
    "ags_render_fwd", "ags_render_bwd", "ags_render_bwd_adam", "ags_bin_records", "ags_adam_step", "ags_pose_step",
    "ags_profile_enable", "ags_profile_read", "ags_profile_reset", "ags_lifecycle_workspace",
    "ags_lifecycle_step", "ags_lifecycle_step_noalloc", "ags_tune", "ags_map_config_default", "ags_map_create", "ags_map_destroy", "ags_map_insert",
    "ags_map_lifecycle", "ags_map_export", "ags_map_read_store", "ags_map_sync", "ags_check_finite",
]


class Config(C.Structure):
    _fields_ = [("alpha_min", C.c_float), ("alpha_max", C.c_float), ("t_min", C.c_float),
                ("blur", C.c_float), ("z_near", C.c_float), ("fov_clamp", C.c_float),
                ("bg", C.c_float * 3), ("tile", C.c_int), ("batch", C.c_int),
                ("px_per_thread", C.c_int), ("batch_bwd", C.c_int), ("px_per_thread_bwd", C.c_int)]


class Views(C.Structure):
    _fields_ = [("n_views", C.c_int), ("width", C.POINTER(C.c_int32)),
                ("height", C.POINTER(C.c_int32)), ("g_begin", C.POINTER(C.c_int32)),
                ("g_end", C.POINTER(C.c_int32))]


class Gaussians(C.Structure):
    _fields_ = [("n", C.c_int32), ("sh_degree", C.c_int32), ("means", C.c_void_p),
                ("log_scales", C.c_void_p), ("quats", C.c_void_p),
                ("opacity_logits", C.c_void_p), ("sh", C.c_void_p)]


class Grads(C.Structure):
    _fields_ = [("means", C.c_void_p), ("log_scales", C.c_void_p), ("quats", C.c_void_p),
                ("opacity_logits", C.c_void_p), ("sh", C.c_void_p), ("pose", C.c_void_p),
                ("accumulate", C.c_int32), ("stat_grad", C.c_void_p), ("stat_count", C.c_void_p)]


class MapConfig(C.Structure):
    _fields_ = [("voxel", C.c_float), ("s_init", C.c_float), ("o_init", C.c_float), ("sh_degree", C.c_int32),
                ("prime", C.c_uint64 * 3), ("max_ids", C.c_int64), ("max_points", C.c_int64), ("tau", C.c_int64)]


class MapCounts(C.Structure):
    _fields_ = [("n_ids", C.c_int64), ("n_resident", C.c_int64), ("n_new", C.c_int64),
                ("n_reloaded", C.c_int64), ("n_evicted", C.c_int64), ("n_offloaded", C.c_int64),
                ("n_retired", C.c_int64)]


class Lifecycle(C.Structure):
    _fields_ = [("do_prune", C.c_int32), ("do_densify", C.c_int32), ("do_reset", C.c_int32),
                ("tau_opa", C.c_float), ("s_min", C.c_float), ("s_max", C.c_float),
                ("grad_threshold", C.c_float), ("kappa", C.c_float), ("s_init", C.c_float),
                ("tau_reset", C.c_float), ("split_scale", C.c_float)]


class TuneEntry(C.Structure):
    _fields_ = [("tile", C.c_int32), ("batch", C.c_int32), ("px_per_thread", C.c_int32),
                ("step_ms", C.c_float), ("raster_fwd_ms", C.c_float), ("raster_bwd_ms", C.c_float),
                ("intersections", C.c_int64)]


class FwdOut(C.Structure):
    _fields_ = [("rgb", C.c_void_p), ("depth", C.c_void_p), ("alpha", C.c_void_p), ("depth_var", C.c_void_p)]


class Upstream(C.Structure):
    _fields_ = [("d_rgb", C.c_void_p), ("d_depth", C.c_void_p), ("d_alpha", C.c_void_p)]


class Loss(C.Structure):
    _fields_ = [("gt_rgb", C.c_void_p), ("mask", C.c_void_p),
                ("l1_count", C.POINTER(C.c_int64)), ("depth_pix", C.c_void_p),
                ("depth_val", C.c_void_p), ("depth_sigma", C.c_void_p),
                ("depth_offsets", C.POINTER(C.c_int64)), ("w_l1", C.c_float),
                ("lambda_lidar", C.c_float), ("sigma_mode", C.c_int32), ("sigma_floor", C.c_float),
                ("ssim_weight", C.c_float)]

SIGMA_FIXED, SIGMA_RENDERED = 0, 1


class Sizes(C.Structure):
    _fields_ = [("saved_bytes", C.c_size_t), ("fwd_ws_bytes", C.c_size_t),
                ("bwd_ws_bytes", C.c_size_t), ("n_pairs", C.c_int64), ("n_pixels", C.c_int64),
                ("n_tiles", C.c_int64), ("tile_bits", C.c_int32), ("off_counters", C.c_size_t),
                ("off_records", C.c_size_t), ("off_pair_count", C.c_size_t),
                ("off_tile_pairs", C.c_size_t), ("off_ranges", C.c_size_t),
                ("off_t_final", C.c_size_t), ("off_last", C.c_size_t),
                ("off_tile_keys", C.c_size_t), ("off_work", C.c_size_t), ("n_work", C.c_int64)]


class Adam(C.Structure):
    _fields_ = [("lr_means", C.c_float), ("lr_log_scales", C.c_float), ("lr_quats", C.c_float),
                ("lr_opacity", C.c_float), ("lr_sh0", C.c_float), ("lr_shrest", C.c_float),
                ("lr_pose", C.c_float), ("beta1", C.c_float), ("beta2", C.c_float),
                ("eps", C.c_float)]


ABI_VERSION = 5  # include/agsplat.h AGS_ABI_VERSION

_lib = None


def load(path: str = LIB_PATH):
    """Load libagsplat.so (once).  Raises ImportError when it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python -c 'import __graft_entry__ as g; g.build()'`"
                          " (no CPU fallback exists)")
    lib = C.CDLL(path)
    lib.ags_version.restype = C.c_int
    if lib.ags_version() != ABI_VERSION:
        raise ImportError(f"{path} implements ABI {lib.ags_version()}, this binding expects {ABI_VERSION}: rebuild it")
    P = C.POINTER
    vp = C.c_void_p
    lib.ags_version.restype = C.c_int
    lib.ags_error_string.restype = C.c_char_p
    lib.ags_error_string.argtypes = [C.c_int]
    lib.ags_last_hip_error.argtypes = [vp]
    lib.ags_config_default.argtypes = [P(Config)]
    lib.ags_config_default.restype = None
    lib.ags_ctx_create.argtypes = [P(vp), C.c_int, P(Config)]
    lib.ags_ctx_destroy.argtypes = [vp]
    lib.ags_ctx_destroy.restype = None
    lib.ags_ctx_set_config.argtypes = [vp, P(Config)]
    lib.ags_buffer_sizes.argtypes = [P(Config), P(Views), C.c_int32, C.c_int32, C.c_int64, P(Sizes)]
    lib.ags_workspace_query.argtypes = [vp, P(Views), C.c_int32, C.c_int32, C.c_int64, P(Sizes)]
    lib.ags_render_fwd.argtypes = [vp, P(Views), P(Gaussians), vp, C.c_int64, P(FwdOut), vp, vp,
                                   C.c_size_t, vp]
    lib.ags_render_bwd.argtypes = [vp, P(Views), P(Gaussians), vp, C.c_int64, P(FwdOut), vp,
                                   P(Upstream), P(Loss), P(Grads), vp, vp, C.c_size_t, vp]
    lib.ags_render_bwd_adam.argtypes = [vp, P(Views), P(Gaussians), vp, C.c_int64, P(FwdOut), vp,
                                        P(Upstream), P(Loss), P(Grads), vp, P(Adam), P(Gaussians), P(Gaussians),
                                        vp, vp, C.c_size_t, vp]
    lib.ags_bin_records.argtypes = [vp, P(Views), C.c_int32, vp, vp, C.c_int64, vp, vp, C.c_size_t, vp]
    lib.ags_adam_step.argtypes = [vp, P(Adam), P(Gaussians), P(Grads), P(Gaussians), P(Gaussians), vp, vp]
    lib.ags_pose_step.argtypes = [vp, P(Adam), vp, C.c_int32, vp, vp, vp, vp, C.c_int32, vp]
    lib.ags_profile_enable.argtypes = [vp, C.c_int]
    lib.ags_profile_read.argtypes = [vp, C.c_int, P(C.c_char_p), P(C.c_double), P(C.c_int64), P(C.c_int)]
    lib.ags_profile_reset.argtypes = [vp]
    lib.ags_map_config_default.argtypes = [P(MapConfig)]
    lib.ags_map_create.argtypes = [vp, P(MapConfig), P(vp)]
    lib.ags_map_destroy.argtypes = [vp]
    lib.ags_map_insert.argtypes = [vp, vp, vp, C.c_int64, C.c_int32, P(Gaussians), P(Gaussians), P(Gaussians), vp,
                                   P(Gaussians), P(Gaussians), P(Gaussians), vp, vp, vp, P(MapCounts), vp]
    lib.ags_map_lifecycle.argtypes = [vp, vp, vp, C.c_int64, P(Gaussians), P(Gaussians), P(Gaussians),
                                      P(Gaussians), P(Gaussians), P(Gaussians), vp, P(MapCounts), vp]
    lib.ags_map_export.argtypes = [vp, vp, vp, vp, vp, vp, C.c_int64, P(C.c_int64), P(C.c_int64)]
    lib.ags_map_read_store.argtypes = [vp, vp, C.c_int64, vp]
    lib.ags_map_sync.argtypes = [vp]
    lib.ags_check_finite.argtypes = [vp, P(Gaussians), vp, vp]
    lib.ags_lifecycle_workspace.argtypes = [C.c_int64, P(C.c_size_t)]
    lib.ags_lifecycle_step.argtypes = [vp, P(Lifecycle), P(Gaussians), P(Gaussians), P(Gaussians), vp, vp, vp,
                                       P(Gaussians), P(Gaussians), P(Gaussians), vp, vp, vp, C.c_size_t, vp]
    lib.ags_lifecycle_step_noalloc.argtypes = [vp, P(Lifecycle), P(Gaussians), P(Gaussians), P(Gaussians), vp, vp,
                                               vp, P(Gaussians), P(Gaussians), P(Gaussians), vp, vp, vp]
    lib.ags_tune.argtypes = [vp, P(Views), P(Gaussians), vp, P(Loss), C.c_int32, C.c_int32, P(Config),
                             P(C.c_float), P(TuneEntry), C.c_int32, P(C.c_int32), vp]
    for name in EXPORTED:
        if lib.ags_version and not hasattr(lib, name):
            raise ImportError(f"libagsplat.so lacks {name}")
    _lib = lib
    return lib


class AgsError(RuntimeError):
    pass


def check(rc: int, what: str = "", ctx=None):
    if rc != AGS_OK:
        lib = load()
        msg = lib.ags_error_string(rc).decode()
        if rc == AGS_ERR_HIP and ctx is not None:
            msg += f" (hipError {lib.ags_last_hip_error(ctx)})"
        raise AgsError(f"{what}: {msg} ({rc})")
