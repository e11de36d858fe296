"""The bit-reproducible reduction (FS_RED_DET).

A (Sec. 3.2 Eq. (7), Sec. 3.3 Eq. (8)) is a sum of weights whose float32
atomic additions round in arrival order. FS_RED_DET adds them as 64-bit
fixed-point integers, so its A must be the same bits on every run, for every
work order, launch shape, lane count, chunking and depth-slab split, while
staying within the acceptance tolerance of the float64 oracle and of the
other reduction strategies."""
import ctypes

import numpy as np
import pytest
import torch

import oracle as O
import scenegen as sg
from paper_2409_08270_amd import _lib as L
from paper_2409_08270_amd.solve import Solver, tiles_of
from tests._parity import REL, ABS, assert_A, assert_labels, log

pytestmark = pytest.mark.gpu


def _scene(E, noise, n=1500, views=3, res=96, seed=0):
    """C1 geometry with masks of a few large regions plus a fraction `noise` of
    pixels relabelled uniformly over E labels (stray labels; E > 64 with noise
    1 sends tiles to the per-pixel path)."""
    sc = sg.make_config("C1", n=n, views=views, res=res)
    rng = np.random.default_rng(100 + E + seed)
    yy, xx = np.mgrid[0:res, 0:res]
    masks = []
    for _ in range(sc.n_views):
        m = ((xx // 24) + 3 * (yy // 24)) % E
        flip = rng.random((res, res)) < noise
        m[flip] = rng.integers(0, E, size=int(flip.sum()))
        masks.append(m.astype(np.uint8))
    sc.masks = masks
    sc.E = E
    return sc


@pytest.fixture(scope="module")
def ctx():
    return L.Context()


def _solve(ctx, ds, prm, chunk, compensated=True, reduction=L.FS_RED_DET):
    out = Solver(ctx, ds, prm).solve(chunk=chunk, reduction=reduction, compensated=compensated)
    torch.cuda.synchronize()
    hi = out["A_hi"].cpu().numpy()
    lo = out["A_lo"].cpu().numpy() if out["A_lo"] is not None else None
    return hi, lo, out["S"].cpu().numpy()


@pytest.mark.parametrize("E,noise", [(2, 0.0), (12, 0.05), (40, 1.0), (100, 1.0)])
def test_det_is_bitwise_repeatable_and_matches_oracle(ctx, E, noise):
    sc = _scene(E, noise)
    ds = L.DeviceScene(sc)
    ref = O.solve64(sc, O.params())
    for chunk in (1, sc.n_views):
        log(f"[det] E={E} noise={noise}: chunk {chunk}, runs under every work order and launch shape")
        hi0, lo0, S0 = _solve(ctx, ds, L.params(), chunk)
        A = hi0.astype(np.float64) + lo0.astype(np.float64)
        assert_A(A, ref["A"], ref["slack"], what=f"det E={E} chunk={chunk}")
        S64, m64 = O.assign64(ref["A"], 0.0)
        assert_labels(S0, S64, m64, ref["A"], A, what=f"det E={E} chunk={chunk}")
        for kw in (dict(), dict(tile_order=1), dict(tile_order=2), dict(persistent=1),
                   dict(tile_order=1, persistent=1), dict(lds_batch=64), dict(count_ops=0)):
            hi, lo, S = _solve(ctx, ds, L.params(**kw), chunk)
            assert np.array_equal(hi.view(np.uint32), hi0.view(np.uint32)), kw
            assert np.array_equal(lo.view(np.uint32), lo0.view(np.uint32)), kw
            assert np.array_equal(S, S0), kw
    # without A_lo: A_hi alone, also the same bits on every run
    h1, _, _ = _solve(ctx, ds, L.params(), sc.n_views, compensated=False)
    h2, _, _ = _solve(ctx, ds, L.params(tile_order=1, persistent=1), sc.n_views, compensated=False)
    assert np.array_equal(h1.view(np.uint32), h2.view(np.uint32))
    assert_A(h1.astype(np.float64), ref["A"], ref["slack"], rel=1e-4, what=f"det E={E} float32 A_hi only")
    st = ctx.status()
    if E > 64:
        assert st["flags"] & L.FS_DEV_MANY_LABELS


def test_det_agrees_with_the_other_strategies(ctx):
    """Strategy equivalence: plain atomics, LDS pre-reduction, LDS + two-sum and
    the fixed-point sums give A within the acceptance tolerance of each other."""
    sc = _scene(12, 0.05, n=2000, views=4, res=128, seed=1)
    ds = L.DeviceScene(sc)
    hi, lo, _ = _solve(ctx, ds, L.params(), 1)
    A_det = hi.astype(np.float64) + lo.astype(np.float64)
    s = np.abs(A_det).sum(axis=1)
    assert s.sum() > 0
    for red, comp in ((L.FS_RED_PLAIN, False), (L.FS_RED_LDS, False), (L.FS_RED_LDS2SUM, True)):
        h, l, _ = _solve(ctx, ds, L.params(), 1, compensated=comp, reduction=red)
        A = h.astype(np.float64) + (l.astype(np.float64) if l is not None else 0.0)
        d = np.abs(A - A_det).sum(axis=1)
        worst = float(np.max(d / np.maximum(s, 1e-300)))
        log(f"[det] reduction {red}: max per-row relative difference from FS_RED_DET {worst:.3e}")
        assert np.all(d <= REL * s + ABS), red


def test_batch_det_is_bitwise_stable_across_launch_settings(ctx):
    """One batch of three scenes with FS_RED_DET: lanes, depth slabs, work order,
    persistent launch, graph or not, and chunk budgets change nothing in A or S."""
    scs = [_scene(E, nz, n=1200 + 300 * i, views=3 + i, res=96, seed=i)
           for i, (E, nz) in enumerate(((2, 0.0), (12, 0.05), (40, 0.3)))]
    dss = [L.DeviceScene(s) for s in scs]
    refs = [O.solve64(s, O.params()) for s in scs]

    def run(prm_kw, **opts):
        b = L.Batch(ctx, dss, L.params(**prm_kw), gammas=[0.0] * len(dss), reduction=L.FS_RED_DET, **opts)
        b.run()
        torch.cuda.synchronize()
        out = [(h.cpu().numpy(), l.cpu().numpy(), S.cpu().numpy()) for h, l, S in zip(b.A_hi, b.A_lo, b.S)]
        b.close()
        return out

    base = run({}, lanes=1)
    for i, (hi, lo, S) in enumerate(base):
        A = hi.astype(np.float64) + lo.astype(np.float64)
        assert_A(A, refs[i]["A"], refs[i]["slack"], what=f"batch det scene {i}")
        S64, m64 = O.assign64(refs[i]["A"], 0.0)
        assert_labels(S, S64, m64, refs[i]["A"], A, what=f"batch det scene {i}")
    settings = [({}, dict(lanes=2)), ({}, dict(lanes=3, depth_slabs=2)), ({"tile_order": 1}, dict(lanes=2)),
                ({"persistent": 1}, dict(lanes=1, depth_slabs=3)), ({}, dict(lanes=1, use_graph=0)),
                ({}, dict(lanes=2, elem_budget=4000, pair_budget=20000))]
    for prm_kw, opts in settings:
        log(f"[det] batch {prm_kw} {opts}")
        got = run(prm_kw, **opts)
        for i, ((h0, l0, S0), (h, l, S)) in enumerate(zip(base, got)):
            assert np.array_equal(h.view(np.uint32), h0.view(np.uint32)), (i, prm_kw, opts)
            assert np.array_equal(l.view(np.uint32), l0.view(np.uint32)), (i, prm_kw, opts)
            assert np.array_equal(S, S0), (i, prm_kw, opts)


def test_det_limits_are_rejected_before_any_work(ctx):
    sc = _scene(2, 0.0, n=500, views=1, res=64)
    ds = L.DeviceScene(sc)
    prm = L.params()
    cams, nv = ds.cams()
    proj = L.Proj(ds.n, nv)
    ctx.fs_project(ds, cams, nv, prm, proj)
    tt = tiles_of(64, 64, prm)
    n = -ctx.fs_bin_sort(proj, cams, prm, L.Bins(1, tt), sync_count=True)
    bins = L.Bins(max(n, 1), tt)
    ctx.fs_bin_sort(proj, cams, prm, bins, sync_count=True)
    A_hi = torch.zeros((ds.n, ds.E), dtype=torch.float32, device="cuda")
    A_lo = torch.zeros_like(A_hi)
    # the call that allocates nothing cannot hold the fixed-point totals
    with pytest.raises(L.FlashSplatError) as e:
        ctx.fs_accumulate_noalloc(proj, bins, cams, ds.masks, ds.E, prm, A_hi, A_lo, L.FS_RED_DET)
    assert e.value.code == L.FS_ERR_ARG
    # more than 2^29 pixels in one call
    big = (L.FsCamera * 1)()
    ctypes.memmove(big, cams, ctypes.sizeof(L.FsCamera))
    big[0].width, big[0].height = 30000, 20000
    with pytest.raises(L.FlashSplatError) as e:
        ctx.fs_accumulate(proj, bins, big, ds.masks, ds.E, prm, A_hi, A_lo, L.FS_RED_DET)
    assert e.value.code == L.FS_ERR_ARG
    torch.cuda.synchronize()
    assert float(A_hi.abs().sum()) == 0.0 and float(A_lo.abs().sum()) == 0.0
