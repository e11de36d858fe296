"""GPU point-prompt propagation against the oracle (Sec. 4.1, supplement
"Binary Mask Association"). Both sides evaluate the distances, depths and
projections in binary32 in the same order, so ids, uv and visibility are
compared exactly."""
import numpy as np
import pytest

import oracle as O
import scenegen as sg
from paper_2409_08270_amd import _lib as L
from tests._parity import log
from tests.test_oracle_prompt import _ray_point, _with_centres

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    return L.Context()


def _prompts(scene, v, n, seed):
    rng = np.random.default_rng(seed)
    W, H = float(scene.W[v]), float(scene.H[v])
    return np.stack([rng.uniform(0, W, n), rng.uniform(0, H, n), rng.uniform(1.0, 6.0, n)], 1).astype(np.float32)


def _check(ctx, scene, ds, v, prompts, k):
    got = ctx.fs_prompt_propagate(ds, v, prompts, k=k)
    ref = O.prompt32(scene, v, prompts, k=k)
    names = ("chosen", "nearest", "uv", "visible")
    for name, a, b in zip(names, got, ref):
        assert a.shape == b.shape, name
        if not np.array_equal(a, b):
            bad = np.argwhere(a != b)
            raise AssertionError(f"{name}: {len(bad)} mismatches, first at {bad[0].tolist()}: "
                                 f"{a[tuple(bad[0])]} vs {b[tuple(bad[0])]} (k={k}, view {v})")
    return got


@pytest.mark.parametrize("k", [1, 10, 32])
def test_small_scene_matches_the_oracle(ctx, k):
    sc = sg.make_config("C1")
    ds = L.DeviceScene(sc)
    for v in (0, 5):
        ch, _, _, vis = _check(ctx, sc, ds, v, _prompts(sc, v, 40, 10 * k + v), k)
        assert (ch >= 0).mean() > 0.9 and vis.mean() > 0.3
    log(f"prompt C1 k={k}: ok")


def test_full_size_scene_matches_the_oracle(ctx):
    sc = sg.make_config("C2")
    ds = L.DeviceScene(sc)
    pr = _prompts(sc, 7, 16, 99)
    _check(ctx, sc, ds, 7, pr, 10)
    log(f"prompt C2 n={sc.n} views={sc.n_views}: ok")


def test_ties_across_workgroups_go_to_the_smaller_index(ctx):
    base = sg.make_config("C1")
    X = _ray_point(base, 0, 64.0, 64.0, 3.0)
    rng = np.random.default_rng(5)
    cen = rng.normal(size=(70000, 3)) * 0.5 + X + 3.0
    # the same centre at indices spread over many workgroups of the search
    dup = [5, 300, 4097, 33333, 69999]
    cen[dup] = X
    cen[[17, 60001]] = _ray_point(base, 0, 64.0, 64.0, 2.9)   # in front of it, both at one depth
    sc = _with_centres(base, cen)
    ds = L.DeviceScene(sc)
    ch, nn, _, _ = _check(ctx, sc, ds, 0, np.array([[64.0, 64.0, 3.0]], np.float32), 7)
    assert nn[0].tolist()[:5] == dup and ch[0] == 17


def test_degenerate_inputs(ctx):
    base = sg.make_config("C1")
    # fewer Gaussians than k, all behind the reference camera
    behind = [_ray_point(base, 1, 64.0, 64.0, -s) for s in (0.5, 1.0, 1.5)]
    sc = _with_centres(base, behind)
    ds = L.DeviceScene(sc)
    ch, nn, uv, vis = _check(ctx, sc, ds, 1, np.array([[64.0, 64.0, 1.0]], np.float32), 5)
    assert ch[0] == -1 and nn[0].tolist() == [0, 1, 2, -1, -1] and not uv.any() and not vis.any()
    # no Gaussians at all
    empty = _with_centres(base, np.zeros((0, 3)))
    de = L.DeviceScene(empty)
    ch, nn, uv, vis = ctx.fs_prompt_propagate(de, 0, [[1.0, 2.0, 3.0]], k=4)
    assert ch.tolist() == [-1] and (nn == -1).all() and not uv.any() and not vis.any()
    # no prompts
    ds1 = L.DeviceScene(base)
    ch, nn, uv, vis = ctx.fs_prompt_propagate(ds1, 0, np.zeros((0, 3)), k=4)
    assert ch.shape == (0,) and uv.shape == (0, base.n_views, 2)


def test_bad_arguments_are_rejected(ctx):
    base = sg.make_config("C1")
    ds = L.DeviceScene(base)
    good = [[10.0, 10.0, 2.0]]
    for kw in (dict(ref_view=-1, prompts=good, k=4), dict(ref_view=base.n_views, prompts=good, k=4),
               dict(ref_view=0, prompts=good, k=0), dict(ref_view=0, prompts=good, k=33),
               dict(ref_view=0, prompts=[[10.0, 10.0, 0.0]], k=4),
               dict(ref_view=0, prompts=[[np.nan, 10.0, 2.0]], k=4)):
        with pytest.raises(RuntimeError):
            ctx.fs_prompt_propagate(ds, **kw)
