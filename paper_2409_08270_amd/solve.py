"""Drivers of the splat-and-accumulate path over the C ABI.

plain:   one fs_project / fs_bin_sort / fs_accumulate per view, with the
         exact pair count read back per view (the paper's per-view scheme).
chunked: the same calls over a chunk of views at once: Gaussians are read once
         per chunk and every kernel covers all tiles of the chunk.

Both add into the same A (A is a sum over views, Eq. (7)), then fs_assign
produces the labels. Only argument marshalling and the loop over views or
chunks live here; all arithmetic runs in the library's kernels.
"""
from __future__ import annotations

import math
from typing import Optional, Sequence

import torch

from . import _lib as L


def tiles_of(W, H, prm) -> int:
    return int(math.ceil(W / prm.tile_w) * math.ceil(H / prm.tile_h))


class Solver:
    """Keeps projection planes and tile lists across calls (grow-only)."""

    def __init__(self, ctx: L.Context, dscene: L.DeviceScene, prm: Optional[L.FsParams] = None,
                 device: str = "cuda"):
        self.ctx = ctx
        self.ds = dscene
        self.prm = prm or L.params()
        self.device = device
        self.proj = None
        self.bins = None
        self.last_pairs = []

    def _proj_for(self, nv):
        if self.proj is None or self.proj.n_views < nv:
            self.proj = L.Proj(self.ds.n, nv, self.device)
        if self.proj.n_views != nv:
            p = L.Proj.__new__(L.Proj)
            p.n, p.n_views = self.ds.n, nv
            p.rec, p.rect = self.proj.rec[:nv], self.proj.rect[:nv]
            p.ntiles, p.flags = self.proj.ntiles[:nv], self.proj.flags[:nv]
            return p
        return self.proj

    def _bins_for(self, capacity, total_tiles):
        if self.bins is None or self.bins.capacity < capacity or self.bins.ranges.shape[0] < total_tiles:
            cap = max(capacity, self.bins.capacity if self.bins else 0)
            tt = max(total_tiles, self.bins.ranges.shape[0] if self.bins else 0)
            self.bins = L.Bins(int(cap * 1.2) + 1024, tt, self.device)
        return self.bins

    def accumulate_views(self, views: Sequence[int], A_hi: torch.Tensor, A_lo: Optional[torch.Tensor],
                         reduction: int = L.FS_RED_AUTO, t_final: Optional[torch.Tensor] = None,
                         n_blend: Optional[torch.Tensor] = None, capacity_hint: Optional[int] = None,
                         acc_events=None):
        """Project, bin and accumulate a contiguous run of views in one set of calls."""
        views = list(views)
        v0, v1 = views[0], views[-1] + 1
        assert views == list(range(v0, v1)), "views must be contiguous"
        cams, nv = self.ds.cams(views)
        proj = self._proj_for(nv)
        prm = self.prm
        self.ctx.fs_project(self.ds, cams, nv, prm, proj)
        total_tiles = sum(tiles_of(int(self.ds.W[v]), int(self.ds.H[v]), prm) for v in views)
        bins = self._bins_for(capacity_hint or 1, total_tiles)
        n = self.ctx.fs_bin_sort(proj, cams, prm, bins, sync_count=True)
        if n < 0:
            bins = self._bins_for(-n, total_tiles)
            n = self.ctx.fs_bin_sort(proj, cams, prm, bins, sync_count=True)
        self.last_pairs.append(n)
        if acc_events is not None:
            acc_events[0].record(self.ctx.stream)
        self.ctx.fs_accumulate(proj, bins, cams, self.ds.masks_of(v0, v1), self.ds.E, prm, A_hi, A_lo,
                               reduction, t_final, n_blend)
        if acc_events is not None:
            acc_events[1].record(self.ctx.stream)
        return n

    def solve(self, chunk: int = 1, reduction: int = L.FS_RED_AUTO, compensated: bool = True,
              gamma: float = 0.0, views: Optional[Sequence[int]] = None, want_margin: bool = True,
              acc_events=None):
        n, E = self.ds.n, self.ds.E
        A_hi = torch.zeros((n, E), dtype=torch.float32, device=self.device)
        A_lo = torch.zeros((n, E), dtype=torch.float32, device=self.device) if compensated else None
        views = list(range(self.ds.n_views)) if views is None else list(views)
        self.last_pairs = []
        for i in range(0, len(views), chunk):
            self.accumulate_views(views[i:i + chunk], A_hi, A_lo, reduction, acc_events=acc_events)
        S = torch.empty((E, n), dtype=torch.uint8, device=self.device)
        margin = torch.empty((E, n), dtype=torch.float32, device=self.device) if want_margin else None
        self.ctx.fs_assign(A_hi, A_lo, n, E, gamma, S, margin)
        return dict(A_hi=A_hi, A_lo=A_lo, S=S, margin=margin, pairs=list(self.last_pairs))
