"""The fewer-masks study (Sec. 4.8 "Ablation study" and the supplement's ablation on the number
of masks, with its count of the objects each Gaussian contributes to).

Every 1/f-th view of a scene is kept, for several f; all the subsets are
solved by one batch (one graph launch, each subset a scene of its own that
shares the Gaussians), and `fs_diagnose` reports, per subset, the objects each
Gaussian contributes to and the overlap of every object's subset with
per-Gaussian reference labels. Only argument marshalling lives here.
"""
from __future__ import annotations

from typing import Dict, Optional, Sequence

import numpy as np
import torch

from . import _lib as L


def subset_views(n_views: int, f: int) -> list:
    """Every f-th view, starting at view 0 (at least one view)."""
    return list(range(0, n_views, max(1, int(f))))


def _iou(overlap: np.ndarray) -> np.ndarray:
    ov = overlap.astype(np.float64)
    union = ov[:, 1] + ov[:, 2] - ov[:, 0]
    with np.errstate(invalid="ignore", divide="ignore"):
        return np.where(union > 0, ov[:, 0] / union, np.nan)


def labels_of(S: torch.Tensor) -> np.ndarray:
    """Per-Gaussian label of an exclusive S [E][n]: the object holding it, -1 if none."""
    s = S.cpu().numpy()
    return np.where(s.any(axis=0), s.argmax(axis=0), -1).astype(np.int32)


def fewer_masks(ctx: L.Context, ds: L.DeviceScene, gt: np.ndarray, fractions: Sequence[int] = (1, 4, 8, 16, 32),
                gamma: float = 0.0, prm: Optional[L.FsParams] = None, rel_eps: float = 0.05) -> Dict[int, dict]:
    """For each f in `fractions` (which must hold 1): the views kept, the IoU of
    every object's subset against `gt` and against the subsets that all views
    give ("agreement"; it needs gamma >= 0, where the subsets are exclusive),
    and the histograms of contributed objects (A above rel_eps of the row) and
    of memberships. Returns {f: report}."""
    fractions = [int(f) for f in fractions]
    if 1 not in fractions:
        raise ValueError("fractions must include 1 (all views)")
    prm = prm or L.params()
    subs = [ds.view_subset(subset_views(ds.n_views, f)) for f in fractions]
    batch = L.Batch(ctx, subs, prm, gammas=[gamma] * len(subs))
    try:
        batch.run()
        dev = ctx.stream.device
        gt_dev = torch.from_numpy(np.ascontiguousarray(gt, dtype=np.int32)).to(dev)
        full = fractions.index(1)
        ref_dev = torch.from_numpy(labels_of(batch.S[full])).to(dev) if gamma >= 0 else None
        out = {}
        for i, f in enumerate(fractions):
            c, m, o = ctx.fs_diagnose(batch.A_hi[i], batch.A_lo[i], batch.S[i], gt_dev, ds.n, ds.E, rel_eps)
            r = {"views": subs[i].n_views, "iou": _iou(o), "contrib_hist": c, "member_hist": m, "overlap": o}
            if ref_dev is not None:
                _, _, o_ref = ctx.fs_diagnose(None, None, batch.S[i], ref_dev, ds.n, ds.E)
                r["agreement"] = _iou(o_ref)
            out[f] = r
        return out
    finally:
        batch.close()
