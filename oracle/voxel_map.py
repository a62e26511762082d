"""Voxel-hashed Gaussian map with a bounded GPU-resident set (oracle; tests only), Sec. III-B
"Incremental Gaussian Mapping" (the voxel key equation) and "Memory Management" (LRU offload
to host memory above a threshold tau, reload when a key is met again).

A plain, slow, dictionary-based statement of what one insertion call, and the map's side of
one lifecycle pass (Sec. III-B "Gaussian Splats Lifecycle Operations"), compute.  The paper
leaves v, P1..P3, tau, the initial splat, the order of the resident set and how pruned and
densified splats relate to the voxel keys unstated; the readings taken here:
  * key: c = floor(p / v) per axis with the division and the floor in float32 (the points'
    precision), k = (c_x P1 + c_y P2 + c_z P3) mod 2^64.  Two voxels whose keys collide are
    merged, as key matching implies.  The key 2^64 - 1 is reserved and replaced by 2^64 - 2.
  * a key names a group of splats: the splat its first point instantiated and that splat's
    descendants by densification (a copy or split child inherits its parent's key and
    last_used); keys are not recomputed as means move.  Pruning retires a splat's id (ids are
    never reused); a key whose group has no live member left is absent from the map.
  * the points of one call are taken in order: a key present in the map marks every live
    member of its group used; a key absent instantiates one splat from the first point
    carrying it: mean p, log-scales ln(s_init) (float32), identity quaternion, logit of
    o_init (float32), SH DC (rgb - 1/2) / C0 in float32 (so that a DC-only splat shows the
    point's colour), the rest of the SH and both Adam moments zero.  New ids count up in
    that order.  A point's id is the smallest live id of its group.
  * every live splat in a group that a point of call t hits has last_used = t.
  * resident set: an ordered list of ids (the rows the GPU holds).  A call appends its new
    splats (id order), then the members of the groups it hit that were offloaded (reloaded
    from the host store, id order); then, while more than tau rows are listed, the least
    recently used ones (smallest last_used; ties: earlier in the list) are offloaded, the
    rest keeping their order.  Offloaded rows keep the values they had on the GPU.
  * a lifecycle pass over the resident set, with one action per row (keep, prune, duplicate,
    split): its output rows, in order, become the resident set; each input's first output
    keeps the input's id, the second output of a duplicated or split input gets a new id
    (counting up in input order); pruned inputs are retired.  The resident set may then
    exceed tau until the next insertion call offloads the excess.
Insertion values are float32 (copies and the float32 initialisation above): the GPU result is
expected bit for bit; the rows a lifecycle pass computes are that pass's (oracle.lifecycle).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .lifecycle import CLONE, PRUNE, SPLIT

EMPTY_KEY = (1 << 64) - 1
MASK64 = (1 << 64) - 1
SH_C0 = 0.28209479177387814   # Y_0^0 = 1 / (2 sqrt(pi))
FIELDS = ("means", "log_scales", "quats", "opacity_logits", "sh")
OFFLOADED, RESIDENT, RETIRED = 0, 1, 2


@dataclass
class VoxelMapParams:
    voxel: float = 0.05
    primes: tuple = (73856093, 19349663, 83492791)
    tau: int = 1 << 20
    sh_degree: int = 3
    s_init: float = 0.005
    o_init: float = 0.1


def voxel_cells(points, voxel):
    """floor(p / v) per axis, division and floor in float32, as int64 (n, 3)."""
    p = np.asarray(points, np.float32)
    return np.floor(p / np.float32(voxel)).astype(np.int64)


def voxel_key(cell, primes):
    """(c_x P1 + c_y P2 + c_z P3) mod 2^64 for one integer cell, with the reserved key moved."""
    k = (int(cell[0]) * primes[0] + int(cell[1]) * primes[1] + int(cell[2]) * primes[2]) & MASK64
    return EMPTY_KEY - 1 if k == EMPTY_KEY else k


def voxel_keys(points, vp: VoxelMapParams):
    """Keys of many points at once (uint64 arithmetic wraps modulo 2^64)."""
    c = voxel_cells(points, vp.voxel).astype(np.uint64)
    P = np.asarray(vp.primes, np.uint64)
    with np.errstate(over="ignore"):
        k = c[:, 0] * P[0] + c[:, 1] * P[1] + c[:, 2] * P[2]
    k[k == np.uint64(EMPTY_KEY)] = np.uint64(EMPTY_KEY - 1)
    return k


def new_splat(point, rgb, vp: VoxelMapParams):
    """Row of a splat instantiated from one point: parameters, Adam moments (zero).  s_init and
    o_init are taken at float32 (the precision a configuration holds them in), their
    logarithms in float64 and rounded to float32."""
    f = np.float32
    K = (vp.sh_degree + 1) ** 2
    sh = np.zeros((K, 3), np.float32)
    sh[0] = (np.asarray(rgb, np.float32) - f(0.5)) / f(SH_C0)
    s0 = float(f(vp.s_init))
    o0 = float(f(vp.o_init))
    p = {"means": np.asarray(point, np.float32).copy(),
         "log_scales": np.full(3, f(np.log(s0)), np.float32),
         "quats": np.array([1, 0, 0, 0], np.float32),
         "opacity_logits": np.array([f(np.log(o0 / (1 - o0)))], np.float32),
         "sh": sh}
    zero = {k: np.zeros_like(a) for k, a in p.items()}
    return {"params": p, "m": zero, "v": {k: a.copy() for k, a in zero.items()}}


@dataclass
class VoxelMap:
    vp: VoxelMapParams
    table: dict = field(default_factory=dict)      # key -> live ids of its group, ascending
    seen: set = field(default_factory=set)         # every key ever entered
    keys: list = field(default_factory=list)       # id -> key
    last_used: list = field(default_factory=list)  # id -> call index
    rows: dict = field(default_factory=dict)       # id -> row, for resident ids (the GPU copy)
    store: dict = field(default_factory=dict)      # id -> row, for offloaded ids (host store)
    retired: set = field(default_factory=set)      # pruned ids
    resident: list = field(default_factory=list)   # ordered resident ids

    def state(self, j):
        return RESIDENT if j in self.rows else OFFLOADED if j in self.store else RETIRED

    def insert(self, points, colors, t):
        """One call: returns dict(point_id, new, reloaded, evicted) (id lists in order)."""
        cells = voxel_cells(points, self.vp.voxel)
        pkeys = [voxel_key(c, self.vp.primes) for c in cells]
        new, hit = [], set()
        for i, k in enumerate(pkeys):
            if k not in self.table:
                j = len(self.keys)
                self.table[k] = [j]
                self.seen.add(k)
                self.keys.append(k)
                self.last_used.append(t)
                self.rows[j] = new_splat(points[i], colors[i], self.vp)
                new.append(j)
            hit.add(k)
        point_id = np.array([self.table[k][0] for k in pkeys], np.int64)
        met = sorted(j for k in hit for j in self.table[k])
        for j in met:
            self.last_used[j] = t
        reloaded = [j for j in met if j in self.store]
        for j in reloaded:
            self.rows[j] = self.store.pop(j)
        listed = self.resident + new + reloaded
        evicted = []
        excess = len(listed) - self.vp.tau
        if excess > 0:
            order = sorted(range(len(listed)), key=lambda q: (self.last_used[listed[q]], q))
            out = set(order[:excess])
            evicted = [listed[q] for q in sorted(out)]
            listed = [j for q, j in enumerate(listed) if q not in out]
            for j in evicted:
                self.store[j] = self.rows.pop(j)
        self.resident = listed
        return {"point_id": point_id, "new": new, "reloaded": reloaded, "evicted": evicted}

    def lifecycle(self, actions, out_params, out_m, out_v):
        """The map's side of one lifecycle pass over the resident set: actions[q] for resident
        row q (oracle.lifecycle's codes); out_*: that pass's output rows (dicts of per-row
        arrays, in output order).  Returns dict(ids, new, retired)."""
        actions = np.asarray(actions)
        assert len(actions) == len(self.resident)
        ids, new, retired = [], [], []
        for q, j in enumerate(self.resident):
            a = int(actions[q])
            if a == PRUNE:
                retired.append(j)
                continue
            ids.append(j)
            if a in (CLONE, SPLIT):
                c = len(self.keys)
                self.keys.append(self.keys[j])
                self.last_used.append(self.last_used[j])
                self.table[self.keys[j]].append(c)
                ids.append(c)
                new.append(c)
        for j in retired:
            group = self.table[self.keys[j]]
            group.remove(j)
            if not group:
                del self.table[self.keys[j]]
            del self.rows[j]
            self.retired.add(j)
        assert len(ids) == len(out_params["means"])
        K = (self.vp.sh_degree + 1) ** 2
        shape = {"means": (3,), "log_scales": (3,), "quats": (4,), "opacity_logits": (1,), "sh": (K, 3)}
        f32 = lambda d, r: {k: np.asarray(d[k][r], np.float32).reshape(shape[k]).copy() for k in FIELDS}
        for r, j in enumerate(ids):
            self.rows[j] = {"params": f32(out_params, r), "m": f32(out_m, r), "v": f32(out_v, r)}
        self.resident = ids
        return {"ids": ids, "new": new, "retired": retired}

    def resident_arrays(self, which="params"):
        """The resident rows stacked in resident order: dict field -> (n, ...) float32."""
        out = {}
        for k in FIELDS:
            rows = [self.rows[j][which][k] for j in self.resident]
            K = (self.vp.sh_degree + 1) ** 2
            empty = {"means": (0, 3), "log_scales": (0, 3), "quats": (0, 4), "opacity_logits": (0, 1),
                     "sh": (0, K, 3)}[k]
            out[k] = np.stack(rows).astype(np.float32) if rows else np.zeros(empty, np.float32)
        out["opacity_logits"] = out["opacity_logits"].reshape(-1)
        return out
