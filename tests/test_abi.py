"""The C-ABI library loads and exports every function include/agsplat.h declares; host-only
calls (version, error strings, defaults, buffer sizing and argument validation) behave as
documented.  No call here touches a GPU."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "agsplat.h")


@pytest.fixture(scope="module")
def lib():
    from paper_2510_26358_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_2510_26358_amd import build
        build.build(verbose=False)
    return _lib.load()


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ags_[a-z_0-9]+)\s*\(", text)))


def test_every_declared_function_is_exported(lib):
    names = declared_functions()
    assert len(names) >= 15
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    from paper_2510_26358_amd import _lib
    assert sorted(_lib.EXPORTED) == names


def test_version_errors_and_defaults(lib):
    from paper_2510_26358_amd import _lib as L
    assert lib.ags_version() == L.ABI_VERSION == 5
    for code in (0, -1, -2, -3, -4, -5):
        assert lib.ags_error_string(code)
    cfg = L.Config()
    lib.ags_config_default(C.byref(cfg))
    assert abs(cfg.alpha_min - 1 / 255) < 1e-9 and abs(cfg.alpha_max - 0.99) < 1e-7
    assert abs(cfg.t_min - 1e-4) < 1e-10 and cfg.tile == 16 and cfg.batch == 256


def _views(ws, hs, g0, g1):
    from paper_2510_26358_amd.rasterizer import ViewSpec
    return ViewSpec(ws, hs, g0, g1)


def test_buffer_sizes_layout(lib):
    from paper_2510_26358_amd import _lib as L
    cfg = L.Config()
    lib.ags_config_default(C.byref(cfg))
    v = _views([1280, 640], [800, 400], [0, 100], [1000, 1000])
    s = L.Sizes()
    assert lib.ags_buffer_sizes(C.byref(cfg), C.byref(v.c), 1000, 3, 12345, C.byref(s)) == 0
    assert s.n_pairs == 1000 + 900
    assert s.n_pixels == 1280 * 800 + 640 * 400
    assert s.n_tiles == 80 * 50 + 40 * 25
    assert s.tile_bits == 13  # 5000 tiles
    offs = [s.off_counters, s.off_records, s.off_pair_count, s.off_tile_pairs, s.off_ranges,
            s.off_t_final, s.off_last]
    assert offs == sorted(offs) and all(o % 256 == 0 for o in offs)
    assert s.off_records - s.off_counters >= 16
    assert s.off_pair_count - s.off_records >= 1900 * 48
    assert s.off_ranges - s.off_tile_pairs >= 12345 * 4
    assert s.saved_bytes >= s.off_last + 4 * s.n_pixels


@pytest.mark.parametrize("case", ["views0", "gend", "gneg", "width0", "tile", "batch", "cap", "deg"])
def test_buffer_sizes_rejects_bad_arguments(lib, case):
    from paper_2510_26358_amd import _lib as L
    cfg = L.Config()
    lib.ags_config_default(C.byref(cfg))
    ws, hs, g0, g1, n, deg, cap = [64], [48], [0], [10], 10, 0, 100
    if case == "gend":
        g1 = [11]
    if case == "gneg":
        g0 = [-1]
    if case == "width0":
        ws = [0]
    if case == "tile":
        cfg.tile = 12
    if case == "batch":
        cfg.batch = 100
    if case == "cap":
        cap = -1
    if case == "deg":
        deg = 4
    v = _views(ws, hs, g0, g1)
    if case == "views0":
        v.c.n_views = 0
    s = L.Sizes()
    assert lib.ags_buffer_sizes(C.byref(cfg), C.byref(v.c), n, deg, cap, C.byref(s)) == L.AGS_ERR_INVALID_ARG


def test_null_context_is_rejected_without_touching_a_device(lib):
    from paper_2510_26358_amd import _lib as L
    assert lib.ags_render_fwd(None, None, None, None, 0, None, None, None, 0, None) == L.AGS_ERR_INVALID_ARG
    s = L.Sizes()
    assert lib.ags_workspace_query(None, None, 0, 0, 0, C.byref(s)) == L.AGS_ERR_INVALID_ARG
    assert lib.ags_profile_enable(None, 1) == L.AGS_ERR_INVALID_ARG


def test_lifecycle_and_map_host_calls(lib):
    """Host-only parts of the lifecycle and voxel-map entry points: workspace sizing, the
    map's defaults, and refusals that need no device."""
    from paper_2510_26358_amd import _lib as L
    nb = C.c_size_t()
    assert lib.ags_lifecycle_workspace(1000, C.byref(nb)) == 0 and nb.value >= 2 * 4 * 1000
    assert lib.ags_lifecycle_workspace(-1, C.byref(nb)) == L.AGS_ERR_INVALID_ARG
    assert lib.ags_lifecycle_step(None, None, None, None, None, None, None, None, None, None, None, None, None,
                                  None, 0, None) == L.AGS_ERR_INVALID_ARG
    cfg = L.MapConfig()
    assert lib.ags_map_config_default(C.byref(cfg)) == 0
    assert abs(cfg.voxel - 0.05) < 1e-7 and list(cfg.prime) == [73856093, 19349663, 83492791]
    assert cfg.tau == 1 << 20 and cfg.max_points == 1 << 20 and cfg.sh_degree == 3
    h = C.c_void_p()
    assert lib.ags_map_create(None, C.byref(cfg), C.byref(h)) == L.AGS_ERR_INVALID_ARG
    assert lib.ags_map_insert(None, None, None, 0, 0, None, None, None, None, None, None, None, None, None, None,
                              None, None) == L.AGS_ERR_INVALID_ARG
    cnt = L.MapCounts()
    assert lib.ags_map_lifecycle(None, None, None, 0, None, None, None, None, None, None, None, C.byref(cnt),
                                 None) == L.AGS_ERR_INVALID_ARG
    assert lib.ags_map_sync(None) == L.AGS_ERR_INVALID_ARG
    assert lib.ags_map_destroy(None) == L.AGS_ERR_INVALID_ARG


def test_tune_and_noalloc_refuse_bad_arguments_without_a_device(lib):
    from paper_2510_26358_amd import _lib as L
    best = L.Config()
    assert lib.ags_tune(None, None, None, None, None, 4, 2, C.byref(best), None, None, 0, None,
                        None) == L.AGS_ERR_INVALID_ARG
    assert lib.ags_lifecycle_step_noalloc(None, None, None, None, None, None, None, None, None, None, None, None,
                                          None, None) == L.AGS_ERR_INVALID_ARG


def test_loss_targets_refuse_lidar_pixels_outside_their_view():
    """The binding checks LiDAR target pixels on the host (where they are host arrays)."""
    import numpy as np
    from paper_2510_26358_amd.rasterizer import LossTargets, ViewSpec
    from tests.oracle_helpers import random_scene
    sc = random_scene(17, n=10, n_views=2)
    views = ViewSpec.from_scene(sc)
    LossTargets.from_scene(sc, views, device="cpu")  # valid targets pass
    for bad in (-1, sc.cameras[1].width * sc.cameras[1].height):
        lid = [dict(d) for d in sc.lidar]
        lid[1]["pix"] = np.append(np.asarray(lid[1]["pix"]), bad).astype(np.int32)
        lid[1]["depth"] = np.append(lid[1]["depth"], 3.0)
        lid[1]["sigma"] = np.append(lid[1]["sigma"], 0.5)
        with pytest.raises(ValueError):
            LossTargets.from_scene(sc, views, device="cpu", lidar=lid)
