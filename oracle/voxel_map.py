"""Voxel-hashed Gaussian map with a bounded GPU-resident set (oracle; tests only), Sec. III-B
"Incremental Gaussian Mapping" (the voxel key equation) and "Memory Management" (LRU offload
to host memory above a threshold tau, reload when a key is met again).

A plain, slow, dictionary-based statement of what one insertion call computes.  The paper
leaves v, P1..P3, tau, the initial splat and the order of the resident set unstated; the
readings (recorded in the design doc):
  * key: c = floor(p / v) per axis with the division and the floor in float32 (the points'
    precision), k = (c_x P1 + c_y P2 + c_z P3) mod 2^64.  Points with equal keys belong to the
    same splat (two voxels whose keys collide are merged, as key matching implies).  The key
    2^64 - 1 is reserved and replaced by 2^64 - 2.
  * the points of one call are taken in order: a key already in the map marks its splat used;
    a new key instantiates one splat from the first point carrying it: mean p, log-scales
    ln(s_init) (float32), identity quaternion, logit of o_init (float32), SH DC
    (rgb - 1/2) / C0 in float32 (so that a DC-only splat shows the point's colour), the rest of
    the SH and both Adam moments zero.  New ids count up in that order.
  * every splat whose key a point of call t carries has last_used = t.
  * resident set: an ordered list of ids (the rows the GPU holds).  A call appends its new
    splats (id order), then the splats it met that were offloaded (reloaded from the host
    store, id order); then, while more than tau rows are listed, the least recently used ones
    (smallest last_used; ties: earlier in the list) are offloaded, the rest keeping their
    order.  Offloaded rows keep the values they had on the GPU.
All values are float32 (copies and the float32 initialisation above): the GPU result is
expected bit for bit.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

EMPTY_KEY = (1 << 64) - 1
MASK64 = (1 << 64) - 1
SH_C0 = 0.28209479177387814   # Y_0^0 = 1 / (2 sqrt(pi))
FIELDS = ("means", "log_scales", "quats", "opacity_logits", "sh")


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
    table: dict = field(default_factory=dict)      # key -> id
    keys: list = field(default_factory=list)       # id -> key
    last_used: list = field(default_factory=list)  # id -> call index
    rows: dict = field(default_factory=dict)       # id -> row, for resident ids (the GPU copy)
    store: dict = field(default_factory=dict)      # id -> row, for offloaded ids (host store)
    resident: list = field(default_factory=list)   # ordered resident ids

    def insert(self, points, colors, t):
        """One call: returns dict(point_id, new, reloaded, evicted) (id lists in order)."""
        cells = voxel_cells(points, self.vp.voxel)
        point_id = np.empty(len(cells), np.int64)
        new, met = [], []
        for i, c in enumerate(cells):
            k = voxel_key(c, self.vp.primes)
            if k not in self.table:
                j = len(self.keys)
                self.table[k] = j
                self.keys.append(k)
                self.last_used.append(t)
                self.rows[j] = new_splat(points[i], colors[i], self.vp)
                new.append(j)
            j = self.table[k]
            point_id[i] = j
            self.last_used[j] = t
            met.append(j)
        reloaded = sorted(set(j for j in met if j in self.store))
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
