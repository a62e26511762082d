"""GPU parity of the voxel-hashed map with its bounded resident set (Sec. III-B, "Incremental
Gaussian Mapping" and "Memory Management") against the oracle, through the C ABI: point ids,
new splats, reloads and least-recently-used offloads, the resident rows (values changed
between calls travel to the host store and back), per-id state and the hash table, all exact;
and, at the bench's size (2^20 points per call), the id mapping and the offload order by
properties and samples."""
import numpy as np
import pytest
import torch

from oracle.voxel_map import FIELDS, VoxelMap as OracleMap, VoxelMapParams, new_splat, voxel_keys

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ras():
    from paper_2510_26358_amd.rasterizer import Rasterizer
    return Rasterizer(0)


def _frame(rng, t, n, spread=1.5, step=0.4, revisit=0.0):
    """Points around a centre moving along x (a row being driven), optionally with a share
    of points from the start of the row (a revisit), and colours in [0, 1]."""
    c = np.array([step * t, 0.0, 0.0])
    pts = c + rng.normal(0, spread, (n, 3))
    k = int(revisit * n)
    if k:
        pts[:k] = rng.normal(0, spread, (k, 3))
    # some points exactly on voxel boundaries and at negative coordinates
    pts[:: 17] = np.round(pts[:: 17] * 4) / 4
    return pts.astype(np.float32), rng.random((n, 3)).astype(np.float32)


def _gpu_arrays(sp, n):
    """Resident SplatParams -> dict field -> (n, ...) numpy in the oracle's layout."""
    return {"means": sp.means.T.cpu().numpy(), "log_scales": sp.log_scales.T.cpu().numpy(),
            "quats": sp.quats.T.cpu().numpy(), "opacity_logits": sp.opacity_logits.cpu().numpy(),
            "sh": sp.sh.permute(2, 0, 1).cpu().numpy()}


def _flat_row(row, which):
    return np.concatenate([np.asarray(row[which][k], np.float32).reshape(-1) for k in FIELDS])


def _compare(gm, om, r_gpu, r_ora, counts, ev_gpu):
    assert np.array_equal(r_gpu.cpu().numpy().astype(np.int64), r_ora["point_id"])
    assert counts["n_new"] == len(r_ora["new"]) and counts["n_reloaded"] == len(r_ora["reloaded"])
    assert counts["n_evicted"] == len(r_ora["evicted"]) and counts["n_ids"] == len(om.keys)
    assert counts["n_resident"] == len(om.resident)
    assert ev_gpu.cpu().numpy().tolist() == r_ora["evicted"]
    assert gm.ids.cpu().numpy().tolist() == om.resident
    for which, sp in (("params", gm.params), ("m", gm.m), ("v", gm.v)):
        g = _gpu_arrays(sp, gm.n)
        o = om.resident_arrays(which)
        for k in FIELDS:
            assert np.array_equal(g[k], o[k]), (which, k)
    ex = gm.export()
    assert ex["keys"].tolist() == om.keys
    assert ex["last_used"].tolist() == om.last_used
    res = np.zeros(len(om.keys), bool)
    res[om.resident] = True
    assert np.array_equal(ex["resident"], res)
    occ = ex["table_keys"] != np.uint64(2 ** 64 - 1)
    assert occ.sum() == len(om.keys)
    pairs = sorted(zip(ex["table_ids"][occ].tolist(), ex["table_keys"][occ].tolist()))
    assert pairs == [(j, k) for j, k in enumerate(om.keys)]
    stored = sorted(om.store)
    if stored:
        rows = gm.read_store(stored)
        for r, j in zip(rows, stored):
            for a, which in enumerate(("params", "m", "v")):
                assert np.array_equal(r[a], _flat_row(om.store[j], which)), (j, which)


def _modify(gm, om, t):
    """Optimiser stand-in: change every resident row on both sides, identically in float32."""
    if gm.n == 0:
        return
    d = np.float32(0.125 * (t + 1))
    gm.params.means.add_(float(d))
    gm.m.sh.add_(1.0)
    gm.v.opacity_logits.mul_(2.0)
    for j in om.resident:
        om.rows[j]["params"]["means"] = (om.rows[j]["params"]["means"] + d).astype(np.float32)
        om.rows[j]["m"]["sh"] = (om.rows[j]["m"]["sh"] + np.float32(1.0)).astype(np.float32)
        om.rows[j]["v"]["opacity_logits"] = (om.rows[j]["v"]["opacity_logits"] * np.float32(2.0)).astype(np.float32)


@pytest.mark.parametrize("seed,deg,tau,voxel,sizes", [
    (401, 1, 300, 0.25, [200, 150, 0, 260, 90, 300, 120, 40, 250]),
    (402, 3, 64, 0.5, [40, 100, 70, 5, 90, 60]),
    (403, 0, 1000, 0.1, [500, 400, 450]),
])
def test_map_sequence_matches_oracle(ras, seed, deg, tau, voxel, sizes):
    from paper_2510_26358_amd.voxel_map import VoxelMap
    rng = np.random.default_rng(seed)
    vp = VoxelMapParams(voxel=voxel, tau=tau, sh_degree=deg, s_init=0.01, o_init=0.2)
    om = OracleMap(vp)
    gm = VoxelMap(ras, voxel=voxel, sh_degree=deg, tau=tau, max_ids=8192, max_points=512, s_init=0.01, o_init=0.2)
    try:
        for t, n in enumerate(sizes):
            pts, cols = _frame(rng, t, n, revisit=0.3 if t % 3 == 2 else 0.0)
            r_ora = om.insert(pts, cols, t)
            r_gpu, counts, ev = gm.insert(torch.from_numpy(pts).cuda(), torch.from_numpy(cols).cuda(), t,
                                          evicted=True)
            torch.cuda.synchronize()
            print("call", t, counts)
            _compare(gm, om, r_gpu, r_ora, counts, ev)
            _modify(gm, om, t)
    finally:
        gm.close()


def test_map_refusals(ras):
    from paper_2510_26358_amd._lib import AgsError
    from paper_2510_26358_amd.voxel_map import VoxelMap
    gm = VoxelMap(ras, voxel=1.0, sh_degree=0, tau=8, max_ids=16, max_points=8)
    try:
        p = torch.zeros(9, 3, device="cuda")
        with pytest.raises(AgsError):                    # more points than max_points
            gm.insert(p, p, 0)
        pts = torch.arange(24, dtype=torch.float32, device="cuda").view(8, 3) * 10
        gm.insert(pts, torch.zeros_like(pts), 1)
        with pytest.raises(AgsError):                    # frames must not go back
            gm.insert(pts, torch.zeros_like(pts), 0)
        pts2 = pts + 1000
        gm.insert(pts2, torch.zeros_like(pts2), 2)       # 16 ids: the map is full
        with pytest.raises(AgsError):                    # capacity: nothing changes
            gm.insert(pts2 + 1000, torch.zeros_like(pts2), 3)
        assert gm.n_ids == 16 and gm.n == 8
        # an empty call keeps everything
        r, c = gm.insert(torch.zeros(0, 3, device="cuda"), torch.zeros(0, 3, device="cuda"), 3)
        assert c["n_resident"] == 8 and c["n_new"] == 0
    finally:
        gm.close()


def test_map_at_full_size(ras):
    """2^20 points per call (four calls along a row, the last revisiting its start), resident
    bound 2^20: point ids equal iff keys equal, new ids in first-occurrence order, the
    resident bound, the LRU property, and sampled rows against the oracle's new splat."""
    from paper_2510_26358_amd.voxel_map import VoxelMap
    rng = np.random.default_rng(404)
    vp = VoxelMapParams(voxel=0.05, tau=1 << 20, sh_degree=3)
    gm = VoxelMap(ras, voxel=vp.voxel, sh_degree=3, tau=vp.tau, max_ids=1 << 23, max_points=1 << 20)
    key_to_id = {}
    try:
        for t in range(4):
            n = 1 << 20
            pts, cols = _frame(rng, t, n, spread=4.0, step=6.0, revisit=0.5 if t == 3 else 0.0)
            pid, counts = gm.insert(torch.from_numpy(pts).cuda(), torch.from_numpy(cols).cuda(), t)
            pid = pid.cpu().numpy().astype(np.int64)
            keys = voxel_keys(pts, vp)
            uk, first, inv = np.unique(keys, return_index=True, return_inverse=True)
            # equal keys <-> equal ids
            ids_of_key = pid[first]
            assert np.array_equal(pid, ids_of_key[inv.reshape(-1)])
            assert len(np.unique(ids_of_key)) == len(uk)
            # known keys keep their ids; new keys are numbered in order of their first point
            known = np.array([int(k) in key_to_id for k in uk])
            if known.any():
                assert all(key_to_id[int(k)] == j for k, j in zip(uk[known], ids_of_key[known]))
            new_first = np.sort(first[~known])
            base = len(key_to_id)
            assert np.array_equal(pid[new_first], base + np.arange(len(new_first)))
            for k, j in zip(uk[~known], ids_of_key[~known]):
                key_to_id[int(k)] = int(j)
            assert counts["n_new"] == len(new_first) and counts["n_ids"] == len(key_to_id)
            assert counts["n_resident"] <= vp.tau
            ex = gm.export()
            last = ex["last_used"]
            assert np.all(last[np.unique(pid)] == t)
            res = ex["resident"]
            if (~res).any():
                assert last[~res].max() <= last[res].min()
            ids = gm.ids.cpu().numpy()
            assert np.array_equal(np.sort(ids), np.nonzero(res)[0])
            # sampled new splats against the oracle's initialisation
            g = _gpu_arrays(gm.params, gm.n)
            row_of = np.full(len(key_to_id), -1)
            row_of[ids] = np.arange(len(ids))
            sample = rng.choice(new_first, 200, replace=False) if len(new_first) >= 200 else new_first
            for i in sample:
                j = pid[i]
                if row_of[j] < 0:
                    continue
                ref = new_splat(pts[i], cols[i], vp)["params"]
                for k in FIELDS:
                    assert np.array_equal(g[k][row_of[j]], np.asarray(ref[k]).reshape(g[k][row_of[j]].shape)), k
            print("call", t, counts)
    finally:
        gm.close()
