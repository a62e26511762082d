"""Pins for the voxel-map oracle (Sec. III-B, "Incremental Gaussian Mapping" and "Memory
Management"): the key's cells at voxel boundaries and for negative coordinates, the key's
linearity in the cell and a constructed key collision, the insertion rules on a hand-built
frame, the DC colour of a new splat against the degree-0 harmonic, LRU offload and reload on
hand-built sequences, the map's side of lifecycle passes (key groups, retired ids, emptied
keys) on a hand-built sequence, and invariants of long random sequences with and without
lifecycle passes."""
import math

import numpy as np

from oracle.lifecycle import CLONE, KEEP, PRUNE, SPLIT
from oracle.voxel_map import (EMPTY_KEY, FIELDS, MASK64, OFFLOADED, RESIDENT, RETIRED, SH_C0, VoxelMap,
                              VoxelMapParams, voxel_cells, voxel_key, voxel_keys)

P = (73856093, 19349663, 83492791)


def test_cells_at_boundaries_and_negative_coordinates():
    v = 0.25  # exactly representable: multiples of v are exact in float32
    pts = np.array([[0.0, 0.25, -0.25], [0.2499999, -1e-7, -0.25000003], [1.0, -1.0, 3.75]], np.float32)
    c = voxel_cells(pts, v)
    assert c.tolist() == [[0, 1, -1], [0, -1, -2], [4, -4, 15]]
    # a coordinate just below a boundary falls in the cell below
    x = np.nextafter(np.float32(0.5), np.float32(0))
    assert voxel_cells(np.array([[x, 0.5, 0]], np.float32), v).tolist() == [[1, 2, 0]]


def test_key_linearity_wraparound_and_a_constructed_collision():
    c = np.array([12, -7, 3])
    k = voxel_key(c, P)
    for axis in range(3):
        e = np.zeros(3, np.int64)
        e[axis] = 1
        assert (voxel_key(c + e, P) - k) % (1 << 64) == P[axis]
    # large cells wrap modulo 2^64 and stay 64-bit
    big = np.array([2 ** 40 + 3, -(2 ** 41), 2 ** 39])
    kb = voxel_key(big, P)
    assert 0 <= kb < (1 << 64) and kb != EMPTY_KEY
    # (c_x + P2, c_y - P1, c_z) has the same key: two voxels whose keys collide are merged
    assert voxel_key(np.array([P[1], -P[0], 0]), P) == voxel_key(np.array([0, 0, 0]), P)
    vp = VoxelMapParams(voxel=1.0, primes=(3, 5, 7), tau=100, sh_degree=0)
    m = VoxelMap(vp)
    pts = np.array([[0.5, 0.5, 0.5], [5.5, -2.5, 0.5], [1.5, 0.5, 0.5]], np.float32)
    r = m.insert(pts, np.full((3, 3), 0.5, np.float32), 0)
    assert r["point_id"].tolist() == [0, 0, 1]
    # the key 2^64 - 1 (the empty-slot mark) is moved to 2^64 - 2
    assert voxel_key(np.array([-1, 0, 0]), (1, 0, 0)) == EMPTY_KEY - 1 == MASK64 - 1


def test_insertion_rules_on_a_hand_built_frame():
    vp = VoxelMapParams(voxel=1.0, tau=10, sh_degree=1, s_init=0.01, o_init=0.2)
    m = VoxelMap(vp)
    pts = np.array([[0.2, 0.2, 0.2], [1.5, 0.1, 0.1], [0.9, 0.9, 0.9], [5.5, 5.5, 5.5], [1.2, 0.3, 0.7]],
                   np.float32)
    rgb = np.array([[1, 0, 0], [0, 1, 0], [0, 0, 1], [0.5, 0.5, 0.5], [1, 1, 1]], np.float32)
    r = m.insert(pts, rgb, 0)
    assert r["point_id"].tolist() == [0, 1, 0, 2, 1]
    assert r["new"] == [0, 1, 2] and r["reloaded"] == [] and r["evicted"] == []
    # splat 0 comes from the first point of its voxel, not the third
    row = m.rows[0]["params"]
    assert np.array_equal(row["means"], pts[0])
    # DC-only colour: Y_0^0 sh_0 + 1/2 gives the point's colour back (Y_0^0 = 1 / (2 sqrt(pi)))
    y00 = 1.0 / (2.0 * math.sqrt(math.pi))
    assert abs(SH_C0 - y00) < 1e-15
    for j, src in ((0, 0), (1, 1), (2, 3)):
        colour = y00 * m.rows[j]["params"]["sh"][0].astype(np.float64) + 0.5
        assert np.allclose(colour, rgb[src], atol=1e-7)
        assert not m.rows[j]["params"]["sh"][1:].any()
    assert np.allclose(np.exp(row["log_scales"]), 0.01, rtol=1e-6)
    assert abs(1 / (1 + math.exp(-float(row["opacity_logits"][0]))) - 0.2) < 1e-6
    assert row["quats"].tolist() == [1, 0, 0, 0]
    assert all(not a.any() for a in m.rows[0]["m"].values()) and all(not a.any() for a in m.rows[0]["v"].values())
    # a second call meets two old voxels and one new one
    r2 = m.insert(np.array([[5.1, 5.9, 5.0], [9.0, 9.0, 9.0], [0.1, 0.1, 0.1]], np.float32),
                  np.zeros((3, 3), np.float32), 1)
    assert r2["point_id"].tolist() == [2, 3, 0]
    assert r2["new"] == [3]
    assert m.last_used == [1, 0, 1, 1]
    assert m.resident == [0, 1, 2, 3]


def _cube(i, v=1.0):
    return np.array([[i * v + 0.5, 0.5, 0.5]], np.float32)


def test_lru_offload_and_reload_on_a_hand_built_sequence():
    vp = VoxelMapParams(voxel=1.0, tau=3, sh_degree=0)
    m = VoxelMap(vp)
    g = np.zeros((1, 3), np.float32)
    for t in range(3):                       # ids 0, 1, 2 at calls 0, 1, 2
        m.insert(_cube(t), g, t)
    assert m.resident == [0, 1, 2] and not m.store
    # values changed on the GPU while resident travel to the host store
    m.rows[0]["params"]["means"] += np.float32(0.125)
    m.rows[0]["m"]["sh"] += np.float32(3.0)
    r = m.insert(np.concatenate([_cube(3), _cube(1)]), np.zeros((2, 3), np.float32), 3)
    # listed [0, 1, 2, 3]; last_used 0:0 1:3 2:2 3:3 -> 0 leaves
    assert r["evicted"] == [0] and m.resident == [1, 2, 3]
    assert m.store[0]["params"]["means"][0] == np.float32(0.625) and m.store[0]["m"]["sh"][0, 0] == 3.0
    # meeting 0 again reloads it after the call's new splats; 2 is then the oldest
    r = m.insert(np.concatenate([_cube(4), _cube(0)]), np.zeros((2, 3), np.float32), 4)
    assert r["new"] == [4] and r["reloaded"] == [0]
    # listed [1, 2, 3, 4, 0] with last_used 3, 2, 3, 4, 4: 2 first, then the earlier of 1 / 3
    assert r["evicted"] == [1, 2] and m.resident == [3, 4, 0]
    assert m.rows[0]["params"]["means"][0] == np.float32(0.625)
    # one call meeting more than tau splats keeps the last ones listed among equals
    r = m.insert(np.concatenate([_cube(i) for i in range(5, 10)]), np.zeros((5, 3), np.float32), 5)
    assert r["new"] == [5, 6, 7, 8, 9]
    assert m.resident == [7, 8, 9]


def test_invariants_of_random_sequences():
    rng = np.random.default_rng(11)
    vp = VoxelMapParams(voxel=0.5, tau=40, sh_degree=1)
    m = VoxelMap(vp)
    seen_keys = set()
    for t in range(30):
        centre = np.array([0.3 * t, 0, 0])
        pts = (centre + rng.normal(0, 1.5, (rng.integers(1, 60), 3))).astype(np.float32)
        r = m.insert(pts, rng.random((len(pts), 3)).astype(np.float32), t)
        cells = voxel_cells(pts, vp.voxel)
        keys = [voxel_key(c, vp.primes) for c in cells]
        seen_keys.update(keys)
        # equal keys <-> equal ids; every id once, resident or stored
        for a in range(len(pts)):
            for b in range(a + 1, len(pts)):
                assert (keys[a] == keys[b]) == (r["point_id"][a] == r["point_id"][b])
        assert len(m.keys) == len(seen_keys)
        assert sorted(m.resident + list(m.store)) == list(range(len(m.keys)))
        assert len(set(m.resident)) == len(m.resident) <= vp.tau
        assert set(m.rows) == set(m.resident)
        # LRU: nothing offloaded was used later than anything resident
        if m.store and m.resident:
            assert max(m.last_used[j] for j in m.store) <= min(m.last_used[j] for j in m.resident)
        # every id met in this call is used now
        assert all(m.last_used[j] == t for j in set(r["point_id"].tolist()))


def test_vectorised_keys_equal_the_per_point_keys():
    rng = np.random.default_rng(5)
    vp = VoxelMapParams(voxel=0.05)
    pts = np.concatenate([rng.normal(0, 30, (500, 3)), rng.normal(0, 1e5, (100, 3))]).astype(np.float32)
    ks = voxel_keys(pts, vp)
    assert ks.dtype == np.uint64
    assert [int(k) for k in ks] == [voxel_key(c, vp.primes) for c in voxel_cells(pts, vp.voxel)]


def _pass_rows(m, actions, mark=100.0):
    """Output rows of a stand-in lifecycle pass over m's resident set: every kept output copies
    its input row; the second output of a duplicated or split input is marked (means[0] +
    mark), so that the test can see where each row went."""
    outs = {w: {k: [] for k in FIELDS} for w in ("params", "m", "v")}
    for q, j in enumerate(m.resident):
        n_out = {KEEP: 1, PRUNE: 0, CLONE: 2, SPLIT: 2}[int(actions[q])]
        for c in range(n_out):
            for w in outs:
                for k in FIELDS:
                    a = np.array(m.rows[j][w][k], np.float32)
                    if c == 1 and w == "params" and k == "means":
                        a[0] += np.float32(mark)
                    outs[w][k].append(a)
    return [{k: np.array(v) for k, v in outs[w].items()} for w in ("params", "m", "v")]


def _lifecycle(m, actions):
    return m.lifecycle(actions, *_pass_rows(m, actions))


def test_lifecycle_passes_on_a_hand_built_sequence():
    vp = VoxelMapParams(voxel=1.0, tau=3, sh_degree=0)
    m = VoxelMap(vp)
    z = lambda n: np.zeros((n, 3), np.float32)
    key0 = voxel_key(voxel_cells(_cube(0), 1.0)[0], vp.primes)
    m.insert(np.concatenate([_cube(0), _cube(1)]), z(2), 0)
    # a duplicate: the copy takes the next id, the parent's key and its last use
    r = _lifecycle(m, [CLONE, KEEP])
    assert r == {"ids": [0, 2, 1], "new": [2], "retired": []}
    assert m.keys[2] == m.keys[0] == key0 and m.last_used[2] == 0 and m.table[key0] == [0, 2]
    assert m.rows[2]["params"]["means"][0] == np.float32(100.5)
    # two new voxels: listed [0, 2, 1, 3, 4], tau 3: the two oldest, 0 and 2, leave
    r = m.insert(np.concatenate([_cube(2), _cube(3)]), z(2), 1)
    assert r["new"] == [3, 4] and r["evicted"] == [0, 2] and m.resident == [1, 3, 4]
    # meeting voxel 0 reloads its whole group; the point's id is the group's smallest
    r = m.insert(_cube(0), z(1), 2)
    assert r["point_id"].tolist() == [0] and r["reloaded"] == [0, 2]
    assert m.last_used[0] == m.last_used[2] == 2
    # listed [1, 3, 4, 0, 2] with last uses 0, 1, 1, 2, 2
    assert r["evicted"] == [1, 3] and m.resident == [4, 0, 2]
    # prune the group's smallest member and split the other: the second child is new
    r = _lifecycle(m, [KEEP, PRUNE, SPLIT])
    assert r == {"ids": [4, 2, 5], "new": [5], "retired": [0]}
    assert m.table[key0] == [2, 5] and m.keys[5] == key0 and m.last_used[5] == 2
    assert m.state(0) == RETIRED and m.state(1) == OFFLOADED and m.state(5) == RESIDENT
    # voxel 0's id is now 2; voxel 1's offloaded splat is reloaded; 4 is the oldest
    r = m.insert(np.concatenate([_cube(0), _cube(1)]), z(2), 3)
    assert r["point_id"].tolist() == [2, 1] and r["new"] == [] and r["reloaded"] == [1]
    assert r["evicted"] == [4] and m.resident == [2, 5, 1]
    # pruning every member empties the key: the next point there makes a new splat
    r = _lifecycle(m, [PRUNE, PRUNE, KEEP])
    assert r == {"ids": [1], "new": [], "retired": [2, 5]} and key0 not in m.table
    r = m.insert(_cube(0), z(1), 4)
    assert r["point_id"].tolist() == [6] and r["new"] == [6] and m.table[key0] == [6]
    assert m.resident == [1, 6] and sorted(m.store) == [3, 4] and m.retired == {0, 2, 5}
    assert m.seen == {voxel_key(voxel_cells(_cube(i), 1.0)[0], vp.primes) for i in range(4)}


def test_invariants_of_random_sequences_with_lifecycle_passes():
    rng = np.random.default_rng(12)
    vp = VoxelMapParams(voxel=0.5, tau=40, sh_degree=0)
    m = VoxelMap(vp)
    for t in range(40):
        if t % 3 == 2 and m.resident:
            act = rng.choice([KEEP, PRUNE, CLONE, SPLIT], len(m.resident), p=[0.5, 0.2, 0.15, 0.15])
            n_ids = len(m.keys)
            r = _lifecycle(m, act)
            assert len(r["ids"]) == int((act != PRUNE).sum() + (act >= CLONE).sum())
            assert r["new"] == list(range(n_ids, len(m.keys)))
        centre = np.array([0.3 * t, 0, 0])
        pts = (centre + rng.normal(0, 1.5, (rng.integers(1, 60), 3))).astype(np.float32)
        r = m.insert(pts, rng.random((len(pts), 3)).astype(np.float32), t)
        keys = [voxel_key(c, vp.primes) for c in voxel_cells(pts, vp.voxel)]
        # groups: the live ids of a key, ascending, each id's key its group's; no empty group
        live = [j for j in range(len(m.keys)) if j not in m.retired]
        assert sorted(j for g in m.table.values() for j in g) == live
        assert all(g and g == sorted(g) and all(m.keys[j] == k for j in g) for k, g in m.table.items())
        # a point's id is its group's smallest; every member of a hit group is used now
        for k, j in zip(keys, r["point_id"].tolist()):
            assert m.table[k][0] == j
            assert all(m.last_used[i] == t for i in m.table[k])
        # every id resident, stored or retired, once
        assert sorted(m.resident + list(m.store) + list(m.retired)) == list(range(len(m.keys)))
        assert len(set(m.resident)) == len(m.resident) <= vp.tau and set(m.rows) == set(m.resident)
        if m.store and m.resident:
            assert max(m.last_used[j] for j in m.store) <= min(m.last_used[j] for j in m.resident)


def test_pruning_every_splat_empties_the_map():
    vp = VoxelMapParams(voxel=1.0, tau=4, sh_degree=0)
    m = VoxelMap(vp)
    z = lambda n: np.zeros((n, 3), np.float32)
    m.insert(np.concatenate([_cube(0), _cube(1), _cube(0)]), z(3), 0)
    r = _lifecycle(m, [PRUNE, PRUNE])
    assert r == {"ids": [], "new": [], "retired": [0, 1]} and not m.table and m.resident == []
    # the same voxels again: new splats, new ids (ids are never reused)
    r = m.insert(np.concatenate([_cube(1), _cube(0)]), z(2), 1)
    assert r["new"] == [2, 3] and r["point_id"].tolist() == [2, 3] and m.resident == [2, 3]
    assert m.state(0) == RETIRED and m.state(2) == RESIDENT
