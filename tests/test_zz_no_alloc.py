"""fs_accumulate_noalloc (the compositing call that allocates nothing; its
workspace is the library's static scratch array) against fs_accumulate on the
same projection and tile lists: A within the acceptance tolerance of A
(1e-4 per row), per-pixel transmittance and blend counts identical, on two
calls in a row, the second with a smaller input; and the size limits are
rejected before any work is enqueued."""
import ctypes

import numpy as np
import pytest
import torch

import oracle as O
import scenegen as sg
from paper_2409_08270_amd import _lib as L
from paper_2409_08270_amd.solve import tiles_of
from tests._parity import REL, ABS, assert_A, log

pytestmark = pytest.mark.gpu


def _lists(ctx, ds, prm):
    """Projection planes and tile lists of every view of a scene (one call each)."""
    cams, nv = ds.cams()
    proj = L.Proj(ds.n, nv)
    ctx.fs_project(ds, cams, nv, prm, proj)
    tt = sum(tiles_of(int(ds.W[v]), int(ds.H[v]), prm) for v in range(nv))
    n = -ctx.fs_bin_sort(proj, cams, prm, L.Bins(1, tt), sync_count=True)
    bins = L.Bins(n, tt)
    assert ctx.fs_bin_sort(proj, cams, prm, bins, sync_count=True) == n
    return cams, nv, proj, bins


def _composite(ctx, fn, ds, cams, proj, bins, prm):
    A_hi = torch.zeros((ds.n, ds.E), dtype=torch.float32, device="cuda")
    A_lo = torch.zeros_like(A_hi)
    px = int(ds.mask_off[-1])
    tf = torch.full((px,), -7.0, dtype=torch.float32, device="cuda")
    nb = torch.full((px,), -7, dtype=torch.int32, device="cuda")
    fn(proj, bins, cams, ds.masks, ds.E, prm, A_hi, A_lo, L.FS_RED_AUTO, tf, nb)
    st = ctx.status()
    A = A_hi.double().cpu().numpy() + A_lo.double().cpu().numpy()
    return A, tf.cpu().numpy(), nb.cpu().numpy(), st


def _check_one(ctx, sc, tile_order, what, persistent=0):
    ds = L.DeviceScene(sc)
    prm = L.params(tile_order=tile_order, persistent=persistent)
    cams, nv, proj, bins = _lists(ctx, ds, prm)
    log(f"[no-alloc] {what}: {sc.n} Gaussians, {nv} views, tile_order {tile_order}, {bins.capacity} pairs")
    A0, tf0, nb0, st0 = _composite(ctx, ctx.fs_accumulate, ds, cams, proj, bins, prm)
    A1, tf1, nb1, st1 = _composite(ctx, ctx.fs_accumulate_noalloc, ds, cams, proj, bins, prm)
    # A: the acceptance bar of A, with fs_accumulate's result as the reference
    d = np.abs(A1 - A0).sum(axis=1)
    s = np.abs(A0).sum(axis=1)
    worst = float(np.max(d / np.maximum(s, 1e-300))) if s.size else 0.0
    log(f"[no-alloc] {what}: max per-row relative difference {worst:.3e}, blends {st1['blends']}")
    assert np.all(d <= REL * s + ABS), what
    assert s.sum() > 0
    # per-pixel outputs and counters come from the same decisions: identical
    assert np.array_equal(tf1.view(np.uint32), tf0.view(np.uint32)), what
    assert np.array_equal(nb1, nb0), what
    for k in ("blends", "evaluated", "bad_labels"):
        assert st1[k] == st0[k], (what, k)
    return ds, A1


def test_noalloc_matches_fs_accumulate_on_two_calls_in_a_row():
    ctx = L.Context()
    big = sg.make_config("C1")                          # 2,000 Gaussians, 8 views 128x128
    small = sg.make_config("C1", n=700, views=3, res=80)
    _, A_big = _check_one(ctx, big, 0, "first call (larger)")
    ds, A_small = _check_one(ctx, small, 0, "second call (smaller)")
    # the smaller call also meets the oracle's bar on its own
    ref = O.solve64(small, O.params())
    assert_A(A_small, ref["A"], ref["slack"], what="no-alloc, smaller call")
    # the other work orders (image order; the XCD-run table built on the device)
    for order in (1, 2):
        _check_one(ctx, small, order, f"smaller call, tile_order {order}")
        _check_one(ctx, big, order, f"larger call, tile_order {order}")
    # the persistent launch, whose work counter also lives in the scratch array
    _check_one(ctx, big, 0, "larger call, persistent", persistent=1)
    _check_one(ctx, small, 0, "smaller call, persistent", persistent=1)
    ctx.close()


def test_noalloc_rejects_sizes_beyond_its_scratch():
    ctx = L.Context()
    lib = L.load()
    prm = L.params()
    dummy = torch.zeros(64, dtype=torch.float32, device="cuda")
    p = ctypes.c_void_p(dummy.data_ptr())
    bins = L.FsBins(p, p, p, 1)
    A = p
    # too many views for the view table
    nv = L.FS_NOALLOC_MAX_VIEWS + 1
    cams = L.cameras(np.tile(np.array([1, 0, 0, 0, 1, 0, 0, 0, 1, 0, 0, 4, 50, 50, 8, 8, 16, 16], np.float32), (nv, 1)))
    proj = L.FsProj(p, p, p, p, 1, nv)
    rc = lib.fs_accumulate_noalloc(ctx.h, ctypes.byref(proj), ctypes.byref(bins), cams, p, 2, ctypes.byref(prm),
                                   A, None, L.FS_RED_AUTO, None)
    assert rc == L.FS_ERR_CAPACITY
    assert b"views" in lib.fs_ctx_last_error(ctx.h)
    # too many tiles: five 8192 x 8192 views hold 5 x 2^18 tiles of 16 x 16 pixels, more than 2^20
    cams = L.cameras(np.tile(np.array([1, 0, 0, 0, 1, 0, 0, 0, 1, 0, 0, 4, 50, 50, 8, 8, 8192, 8192], np.float32),
                             (5, 1)))
    proj = L.FsProj(p, p, p, p, 1, 5)
    rc = lib.fs_accumulate_noalloc(ctx.h, ctypes.byref(proj), ctypes.byref(bins), cams, p, 2, ctypes.byref(prm),
                                   A, None, L.FS_RED_AUTO, None)
    assert rc == L.FS_ERR_CAPACITY
    assert b"tiles" in lib.fs_ctx_last_error(ctx.h)
    # nothing was enqueued: the status holds no latched condition
    st = ctx.status()
    assert st["blends"] == 0 and st["flags"] == 0
    ctx.close()
