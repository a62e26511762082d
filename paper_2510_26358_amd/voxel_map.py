"""Voxel-hashed Gaussian map with a bounded GPU-resident set (Sec. III-B, "Incremental
Gaussian Mapping" and "Memory Management", with the lifecycle operations over its splats),
over the ags_map_* calls of libagsplat.

Argument marshalling only: every step runs in the library (the rules are stated with
ags_map_insert and ags_map_lifecycle in include/agsplat.h).  The map keeps two buffer sets
for the resident set (parameters, Adam moments, ids) of at least `tau` rows each and
alternates between them; `params`, `m`, `v` and `ids` are views of the current set, packed
with row stride `n`, ready for the rasteriser and the optimiser (which may change their
values in place, not their rows).  A lifecycle pass writes its output rows into a scratch
set, which ags_map_lifecycle packs into the other set (both grown to twice the resident rows
when needed).
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import _lib as L
from .rasterizer import Rasterizer, SplatParams, _stream

FIELD_ROWS = (3, 3, 4, 1)   # means, log-scales, quaternion, logit; then 3 (deg + 1)^2 SH rows


class VoxelMap:
    def __init__(self, ras: Rasterizer, voxel=0.05, sh_degree=3, tau=1 << 20, max_ids=1 << 22,
                 max_points=1 << 20, s_init=0.005, o_init=0.1, primes=(73856093, 19349663, 83492791)):
        self.lib, self.ctx, self.device = ras.lib, ras.ctx, ras.device
        cfg = L.MapConfig()
        L.check(self.lib.ags_map_config_default(C.byref(cfg)), "ags_map_config_default")
        cfg.voxel, cfg.s_init, cfg.o_init, cfg.sh_degree = voxel, s_init, o_init, sh_degree
        for k in range(3):
            cfg.prime[k] = int(primes[k])
        cfg.max_ids, cfg.max_points, cfg.tau = max_ids, max_points, tau
        self.cfg = cfg
        self.sh_degree, self.tau, self.max_points = sh_degree, tau, max_points
        self.K = (sh_degree + 1) ** 2
        self.F = 11 + 3 * self.K
        h = C.c_void_p()
        L.check(self.lib.ags_map_create(self.ctx, C.byref(cfg), C.byref(h)), "ags_map_create", self.ctx)
        self.h = h
        self.bufs = [self._alloc(tau) for _ in range(2)]
        self.cur = 0
        self.n = 0
        self.n_ids = 0
        self.n_offloaded = 0
        self.scratch = None

    def _alloc(self, cap):
        rows = list(FIELD_ROWS) + [3 * self.K]
        arrays = [[torch.zeros(r * cap, device=self.device) for r in rows] for _ in range(3)]
        return {"arrays": arrays, "ids": torch.zeros(cap, dtype=torch.int32, device=self.device), "cap": cap}

    def _gaussians(self, buf, t, n):
        a = buf["arrays"][t]
        return L.Gaussians(n, self.sh_degree, *[x.data_ptr() for x in a])

    def _view(self, t, buf=None, n=None):
        a = (buf or self.bufs[self.cur])["arrays"][t]
        n = self.n if n is None else n
        return SplatParams(a[0][:3 * n].view(3, n), a[1][:3 * n].view(3, n), a[2][:4 * n].view(4, n), a[3][:n],
                           a[4][:3 * self.K * n].view(self.K, 3, n), self.sh_degree)

    @property
    def params(self) -> SplatParams:
        return self._view(0)

    @property
    def m(self) -> SplatParams:
        return self._view(1)

    @property
    def v(self) -> SplatParams:
        return self._view(2)

    @property
    def ids(self) -> torch.Tensor:
        return self.bufs[self.cur]["ids"][:self.n]

    def insert(self, points: torch.Tensor, colors: torch.Tensor, frame: int, evicted: bool = False):
        """points, colors: (M, 3) float32 on the device.  Returns (point_id (M,) int32, counts dict
        [, evicted ids (n_evicted,) int32])."""
        M = int(points.shape[0])
        assert points.is_contiguous() and colors.is_contiguous() and points.dtype == torch.float32
        src, dst = self.bufs[self.cur], self.bufs[1 - self.cur]
        ins = [self._gaussians(src, t, self.n) for t in range(3)]
        outs = [self._gaussians(dst, t, dst["cap"]) for t in range(3)]
        point_id = torch.empty(max(M, 1), dtype=torch.int32, device=self.device)
        n_ev = max(M, self.n + M + self.n_offloaded - self.tau, 1)
        ev = torch.empty(n_ev, dtype=torch.int32, device=self.device) if evicted else None
        cnt = L.MapCounts()
        rc = self.lib.ags_map_insert(self.h, points.data_ptr() if M else None, colors.data_ptr() if M else None, M,
                                     int(frame), C.byref(ins[0]), C.byref(ins[1]), C.byref(ins[2]),
                                     src["ids"].data_ptr(), C.byref(outs[0]), C.byref(outs[1]), C.byref(outs[2]),
                                     dst["ids"].data_ptr(), point_id.data_ptr(),
                                     ev.data_ptr() if ev is not None else None, C.byref(cnt), _stream())
        L.check(rc, "ags_map_insert", self.ctx)
        counts = self._advance(cnt)
        res = (point_id[:M], counts)
        return res + (ev[:counts["n_evicted"]],) if evicted else res

    def _advance(self, cnt):
        self.cur = 1 - self.cur
        self.n = int(cnt.n_resident)
        self.n_ids = int(cnt.n_ids)
        self.n_offloaded = int(cnt.n_offloaded)
        return {k: int(getattr(cnt, k)) for k, _ in L.MapCounts._fields_}

    def lifecycle(self, ras: Rasterizer, lp, stats=None, noise=None):
        """One lifecycle pass (prune / densify / reset, ags_lifecycle_step) over the resident
        set, then the map's side of it (ags_map_lifecycle).  stats: (grad_accum, count) per
        resident row, noise: (n, 2, 3) standard normals, as Rasterizer.lifecycle takes them.
        Returns (actions (n,) uint8, counts dict, the pass's own output count)."""
        n = self.n
        if self.scratch is None or self.scratch["cap"] < 2 * n:
            self.scratch = self._alloc(max(2 * n, 1))
        if self.bufs[1 - self.cur]["cap"] < 2 * n:
            self.bufs[1 - self.cur] = self._alloc(max(2 * n, self.tau))
        sc, dst = self.scratch, self.bufs[1 - self.cur]
        outs = [self._view(t, sc, sc["cap"]) for t in range(3)]
        n_out = torch.zeros(1, dtype=torch.int32, device=self.device)
        actions = torch.empty(max(n, 1), dtype=torch.uint8, device=self.device)
        ws = torch.empty(max(ras.lifecycle_workspace(n), 1), dtype=torch.uint8, device=self.device)
        ras.lifecycle_into(self.params, self.m, self.v, lp, outs, n_out, actions, ws, stats=stats, noise=noise)
        rows = [self._gaussians(sc, t, sc["cap"]) for t in range(3)]
        dsts = [self._gaussians(dst, t, dst["cap"]) for t in range(3)]
        cnt = L.MapCounts()
        rc = self.lib.ags_map_lifecycle(self.h, self.ids.data_ptr() if n else None,
                                        actions.data_ptr() if n else None, n, C.byref(rows[0]), C.byref(rows[1]),
                                        C.byref(rows[2]), C.byref(dsts[0]), C.byref(dsts[1]), C.byref(dsts[2]),
                                        dst["ids"].data_ptr(), C.byref(cnt), _stream())
        L.check(rc, "ags_map_lifecycle", self.ctx)
        return actions[:n], self._advance(cnt), int(n_out.item())

    def sync(self):
        """Wait until the host store holds the rows the last insertion offloaded."""
        L.check(self.lib.ags_map_sync(self.h), "ags_map_sync", self.ctx)

    def export(self):
        """Per-id keys (uint64), last_used (int32), state (uint8: 0 offloaded, 1 resident,
        2 retired) and resident (bool), and the table's keys / values."""
        n_ids, n_slots = C.c_int64(), C.c_int64()
        L.check(self.lib.ags_map_export(self.h, None, None, None, None, None, 0, C.byref(n_ids), C.byref(n_slots)),
                "ags_map_export", self.ctx)
        I, S = int(n_ids.value), int(n_slots.value)
        keys = np.zeros(max(I, 1), np.uint64)
        last = np.zeros(max(I, 1), np.int32)
        res = np.zeros(max(I, 1), np.uint8)
        tk = np.zeros(S, np.uint64)
        ti = np.zeros(S, np.int32)
        L.check(self.lib.ags_map_export(self.h, keys.ctypes.data, last.ctypes.data, res.ctypes.data, tk.ctypes.data,
                                        ti.ctypes.data, S, None, None), "ags_map_export", self.ctx)
        return {"keys": keys[:I], "last_used": last[:I], "state": res[:I].copy(), "resident": res[:I] == 1,
                "table_keys": tk, "table_ids": ti}

    def read_store(self, ids) -> np.ndarray:
        """Rows (n, 3, F) of offloaded ids from the host store: parameters, m, v."""
        ids = np.ascontiguousarray(ids, np.int32)
        rows = np.zeros((max(len(ids), 1), 3 * self.F), np.float32)
        L.check(self.lib.ags_map_read_store(self.h, ids.ctypes.data, len(ids), rows.ctypes.data),
                "ags_map_read_store", self.ctx)
        return rows[:len(ids)].reshape(-1, 3, self.F)

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            self.lib.ags_map_destroy(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
