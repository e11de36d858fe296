"""The batched solve (fs_batch_*): many scenes of uneven size, every view, the
assignment included, in one hipGraph launch. Checked against the oracle per
scene, against itself across chunkings and graph replays, and against the
single-scene calls."""
import numpy as np
import pytest
import torch

import oracle as O
import scenegen as sg
from paper_2409_08270_amd import _lib as L
from paper_2409_08270_amd.solve import Solver
from tests._parity import assert_A, assert_labels, log

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    return L.Context()


def _uneven_scenes():
    """Three small scenes: different Gaussian counts, view counts, image sizes
    (one ragged) and class counts."""
    a = sg.make_config("C1", n=900, views=2, res=64)
    b = sg.make_config("C1", seed=11, n=2300, views=4, res=100)
    c = sg.make_config("C1", seed=12, n=1500, views=3, res=80)
    rng = np.random.default_rng(7)
    # scene c: 5 classes in blocks, plus 1% relabels
    for i, m in enumerate(c.masks):
        base = ((np.arange(80)[None, :] // 20) + (np.arange(80)[:, None] // 40) + i) % 5
        noise = rng.random(m.shape) < 0.01
        c.masks[i] = np.where(noise, rng.integers(0, 5, size=m.shape), base).astype(np.uint8)
    c.E = 5
    return [a, b, c]


def _A(batch, i):
    A = batch.A_hi[i].double()
    if batch.A_lo[i] is not None:
        A = A + batch.A_lo[i].double()
    return A.cpu().numpy()


def test_multi_scene_batch_matches_the_oracle(ctx):
    scenes = _uneven_scenes()
    gammas = [0.0, 0.3, -0.2]
    dss = [L.DeviceScene(s) for s in scenes]
    log("[batch] 3 scenes, one graph")
    b = L.Batch(ctx, dss, L.params(), gammas=gammas, want_margin=True, lanes=1)
    b.run()
    torch.cuda.synchronize()
    st = ctx.status()
    info = b.info()
    assert info["n_chunks"] == 1 and info["n_views"] == 9
    blends = 0
    for i, sc in enumerate(scenes):
        ref = O.solve64(sc, O.params())
        blends += ref["blends"]
        assert_A(_A(b, i), ref["A"], ref["slack"], what=f"batch scene {i}")
        S64, m64 = O.assign64(ref["A"], gammas[i])
        assert_labels(b.S[i].cpu().numpy(), S64, m64, ref["A"], _A(b, i), what=f"batch scene {i}")
        # margins are |a_n - o_n - gamma| of the normalised sums (Eq. (8)), within the A tolerance
        mg = b.margin[i].cpu().numpy()
        assert np.all(mg >= 0)
        assert np.quantile(np.abs(mg - m64), 0.99) <= 1e-3
    assert abs(st["blends"] - blends) <= 1e-3 * blends


def test_chunked_batch_equals_one_chunk(ctx):
    scenes = _uneven_scenes()
    dss = [L.DeviceScene(s) for s in scenes]
    one = L.Batch(ctx, dss, L.params(), lanes=1)
    one.run()
    # budgets that force a chunk boundary inside scenes
    many = L.Batch(ctx, dss, L.params(), elem_budget=5000, pair_budget=20000)
    many.run()
    torch.cuda.synchronize()
    ctx.status()
    assert many.info()["n_chunks"] >= 3
    assert many.info()["pairs"] == one.info()["pairs"]
    for i in range(len(scenes)):
        a, c = _A(one, i), _A(many, i)
        d = np.abs(a - c).sum(1)
        s = np.abs(a).sum(1)
        assert np.all(d <= 1e-5 * s + 1e-9), f"scene {i}"
        # summation order differs between chunkings: labels may differ only where the margin is in the last bits
        diff = one.S[i].cpu().numpy() != many.S[i].cpu().numpy()
        assert diff.sum() <= 2, f"scene {i}: {int(diff.sum())} label flips"


def test_graph_replays_match_the_eager_enqueue(ctx):
    scenes = _uneven_scenes()[:2]
    dss = [L.DeviceScene(s) for s in scenes]
    eager = L.Batch(ctx, dss, L.params(), use_graph=0)
    eager.run()
    torch.cuda.synchronize()
    want = [_A(eager, i) for i in range(2)]
    want_S = [eager.S[i].cpu().numpy() for i in range(2)]
    g = L.Batch(ctx, dss, L.params(), use_graph=1)
    for rep in range(4):
        # unrelated eager work and synchronisations between the replays
        x = torch.randn(1 << 20, device="cuda")
        (x * 2).sum().item()
        g.run()
        torch.cuda.synchronize()
        for i in range(2):
            a = _A(g, i)
            d = np.abs(a - want[i]).sum(1)
            s = np.abs(want[i]).sum(1)
            assert np.all(d <= 1e-5 * s + 1e-9), f"replay {rep} scene {i}"
            # labels differ only where the bias-free margin sits in the last bits
            diff = g.S[i].cpu().numpy() != want_S[i]
            assert diff.sum() <= 2, f"replay {rep} scene {i}: {int(diff.sum())} label flips"
    st = ctx.status()
    assert st["flags"] & (L.FS_DEV_PAIR_OVERFLOW | L.FS_DEV_BAD_LABEL) == 0


def test_accumulating_runs_add_up(ctx):
    sc = sg.make_config("C1", n=1200, views=3, res=72)
    ds = L.DeviceScene(sc)
    b = L.Batch(ctx, [ds], L.params(), zero_accumulators=0, want_labels=False)
    b.run()
    torch.cuda.synchronize()
    once = _A(b, 0)
    b.run()
    torch.cuda.synchronize()
    twice = _A(b, 0)
    d = np.abs(twice - 2 * once).sum(1)
    assert np.all(d <= 1e-5 * np.abs(once).sum(1) + 1e-9)


def test_batch_equals_single_scene_calls(ctx):
    sc = sg.make_config("C1", n=2000, views=5, res=96)
    ds = L.DeviceScene(sc)
    b = L.Batch(ctx, [ds], L.params(), gammas=[0.2])
    b.run()
    out = Solver(ctx, ds).solve(chunk=5, gamma=0.2)
    torch.cuda.synchronize()
    ctx.status()
    a = _A(b, 0)
    c = (out["A_hi"].double() + out["A_lo"].double()).cpu().numpy()
    d = np.abs(a - c).sum(1)
    assert np.all(d <= 1e-5 * np.abs(c).sum(1) + 1e-9)


def test_batch_with_an_empty_scene(ctx):
    empty = sg.make_custom(np.zeros((0, 3)), np.zeros((0, 3)), np.zeros((0, 4)), np.zeros(0),
                           [(np.eye(3), np.zeros(3))], W=40, H=24)
    sc = sg.make_config("C1", n=800, views=2, res=64)
    dss = [L.DeviceScene(empty), L.DeviceScene(sc)]
    b = L.Batch(ctx, dss, L.params())
    b.run()
    torch.cuda.synchronize()
    ctx.status()
    ref = O.solve64(sc, O.params())
    assert_A(_A(b, 1), ref["A"], ref["slack"], what="next to an empty scene")


def test_batch_rejects_bad_arguments(ctx):
    sc = sg.make_config("C1", n=300, views=1, res=32)
    ds = L.DeviceScene(sc)
    with pytest.raises(L.FlashSplatError):
        L.Batch(ctx, [ds], L.params(tile_order=2))
    with pytest.raises(L.FlashSplatError):
        L.Batch(ctx, [ds], L.params(), gammas=[1.5])
    with pytest.raises(L.FlashSplatError):
        L.Batch(ctx, [ds], L.params(), compensated=False, reduction=L.FS_RED_LDS2SUM)


def test_depth_slabs_give_the_single_pass_result(ctx):
    """Front-to-back depth slabs (tiles whose pixels have finished get no later pairs)
    composite the same weights as one pass over the full lists."""
    scenes = _uneven_scenes()
    dss = [L.DeviceScene(s) for s in scenes]
    ctx.status()
    one = L.Batch(ctx, dss, L.params(), depth_slabs=1)
    one.run()
    torch.cuda.synchronize()
    st1 = ctx.status()
    assert st1["pairs_emitted"] == one.info()["pairs"]
    for S in (2, 3, 4):
        b = L.Batch(ctx, dss, L.params(), depth_slabs=S)
        b.run()
        torch.cuda.synchronize()
        st = ctx.status()
        log(f"[slabs] S={S}: pairs emitted {st['pairs_emitted']} of {one.info()['pairs']}; blends {st['blends']} "
            f"vs {st1['blends']}")
        assert st["pairs_emitted"] <= st1["pairs_emitted"]
        assert abs(st["blends"] - st1["blends"]) <= 1e-4 * st1["blends"]
        assert st["bad_labels"] == st1["bad_labels"]
        for i in range(len(scenes)):
            a, c = _A(one, i), _A(b, i)
            d = np.abs(a - c).sum(1)
            assert np.all(d <= 1e-5 * np.abs(a).sum(1) + 1e-9), f"S={S} scene {i}"


def test_uncounted_batch_gives_the_same_result(ctx):
    # count_ops = 0 drops only the evaluation/blend counters of the compositing
    scenes = _uneven_scenes()
    dss = [L.DeviceScene(s) for s in scenes]
    out = {}
    for count in (1, 0):
        b = L.Batch(ctx, dss, L.params(count_ops=count), gammas=[0.0, 0.3, -0.2], want_margin=True)
        ctx.status()
        b.run()
        torch.cuda.synchronize()
        st = ctx.status()
        out[count] = ([_A(b, i) for i in range(3)], [b.S[i].cpu().numpy() for i in range(3)], st)
        b.close()
    (A1, S1, st1), (A0, S0, st0) = out[1], out[0]
    assert st1["blends"] > 0 and st1["evaluated"] >= st1["blends"]
    assert st0["blends"] == 0 and st0["evaluated"] == 0
    assert st0["pairs_emitted"] == st1["pairs_emitted"] and st0["wave_steps"] == st1["wave_steps"]
    for i in range(3):
        # the atomics' order may differ between runs; A_hi + A_lo agrees to about one rounding
        assert np.allclose(A0[i], A1[i], rtol=1e-6, atol=1e-9)
        assert np.array_equal(S0[i], S1[i])
    with pytest.raises(RuntimeError):
        L.Batch(ctx, dss, L.params(count_ops=2))


def test_depth_slabs_on_the_global_key_sort(ctx):
    """Depth slabs where the pairs cannot be packed into one word (3M Gaussians need
    22 id bits, 1297x840 views 13 tile bits): the (tile, depth) key sort with tiles
    that finished skipped in later slabs gives the single-pass result."""
    sc = sg.make_config("C4", views=2)
    ds = L.DeviceScene(sc)
    out = {}
    for S in (1, 2):
        b = L.Batch(ctx, [ds], L.params(), gammas=[0.0], depth_slabs=S)
        ctx.status()
        b.run()
        torch.cuda.synchronize()
        st = ctx.status()
        out[S] = (_A(b, 0), b.S[0].cpu().numpy(), st)
        if S == 1:
            inf, _, _, _ = b.chunk_lists(0)
            assert inf["packed"] == 0
        b.close()
    (a1, s1, st1), (a2, s2, st2) = out[1], out[2]
    log(f"[slabs, global keys] pairs emitted {st2['pairs_emitted']} of {st1['pairs_emitted']}")
    assert st2["pairs_emitted"] < st1["pairs_emitted"]
    assert abs(st2["blends"] - st1["blends"]) <= 1e-4 * st1["blends"]
    d = np.abs(a1 - a2).sum(1)
    assert np.all(d <= 1e-5 * np.abs(a1).sum(1) + 1e-9)
    assert (s1 != s2).sum() <= 2


@pytest.mark.parametrize("slabs", [1, 2])
def test_grown_inputs_overflow_is_latched(ctx, slabs):
    # The plan (pair capacities, per-view sort segments) is exact for the inputs
    # at creation. Scaling the Gaussians up afterwards makes every view need more
    # pairs: the excess must be dropped and latched, never written out of bounds,
    # and restoring the inputs restores the result (one slab and two slabs, both
    # on the packed per-view pair sort).
    sc = sg.make_config("C1", n=5000, views=3, res=96)
    ds = L.DeviceScene(sc)
    b = L.Batch(ctx, [ds], L.params(), depth_slabs=slabs)
    ctx.status()
    b.run()
    torch.cuda.synchronize()
    st = ctx.status()
    assert st["flags"] & L.FS_DEV_PAIR_OVERFLOW == 0 and st["pairs_dropped"] == 0
    A0, S0 = _A(b, 0), b.S[0].cpu().numpy()
    scales = [ds.arrays[k].clone() for k in (7, 8, 9)]
    for k in (7, 8, 9):
        ds.arrays[k].mul_(6.0)
    b.run()
    torch.cuda.synchronize()
    st = ctx.status()
    log(f"[batch overflow slabs={slabs}] dropped {st['pairs_dropped']} flags {st['flags']}")
    assert st["flags"] & L.FS_DEV_PAIR_OVERFLOW and st["pairs_dropped"] > 0
    for k, s0 in zip((7, 8, 9), scales):
        ds.arrays[k].copy_(s0)
    b.run()
    torch.cuda.synchronize()
    st = ctx.status()
    assert st["flags"] & L.FS_DEV_PAIR_OVERFLOW == 0
    assert np.allclose(_A(b, 0), A0, rtol=1e-6, atol=1e-9) and np.array_equal(b.S[0].cpu().numpy(), S0)
    b.close()


@pytest.mark.parametrize("use_graph", [1, 0])
def test_lanes_give_the_one_lane_result(ctx, use_graph):
    # chunks on two to four lanes (streams) add into the same accumulators
    scenes = _uneven_scenes()
    dss = [L.DeviceScene(s) for s in scenes]
    one = L.Batch(ctx, dss, L.params(), gammas=[0.0, 0.3, -0.2], lanes=1, use_graph=use_graph)
    one.run()
    torch.cuda.synchronize()
    ctx.status()
    assert one.info()["n_chunks"] == 1
    for lanes in (0, 2, 3, 4):
        b = L.Batch(ctx, dss, L.params(), gammas=[0.0, 0.3, -0.2], lanes=lanes, use_graph=use_graph)
        for _ in range(2):  # replays start from zero again
            b.run()
        torch.cuda.synchronize()
        st = ctx.status()
        assert st["flags"] == 0
        assert b.info()["n_chunks"] >= (lanes if lanes else 2)
        assert b.info()["pairs"] == one.info()["pairs"]
        for i in range(len(scenes)):
            a, c = _A(one, i), _A(b, i)
            d = np.abs(a - c).sum(1)
            s = np.abs(a).sum(1)
            assert np.all(d <= 1e-5 * s + 1e-9), f"lanes {lanes} scene {i}"
            diff = one.S[i].cpu().numpy() != b.S[i].cpu().numpy()
            assert diff.sum() <= 2, f"lanes {lanes} scene {i}: {int(diff.sum())} label flips"
        b.close()
    with pytest.raises(RuntimeError):
        L.Batch(ctx, dss, L.params(), lanes=5)


@pytest.mark.parametrize("persistent,lds_batch,lanes", [(1, 0, 2), (1, 64, 1), (0, 32, 2), (0, 128, 3)])
def test_launch_shapes_match_the_oracle(ctx, persistent, lds_batch, lanes):
    # the persistent compositing launch (resident workgroups pulling tiles from a
    # device counter) and smaller LDS batches give the oracle's A and labels,
    # in the graph and replayed
    scenes = _uneven_scenes()
    dss = [L.DeviceScene(s) for s in scenes]
    prm = L.params(persistent=persistent, lds_batch=lds_batch)
    b = L.Batch(ctx, dss, prm, gammas=[0.0, 0.3, -0.2], lanes=lanes)
    for _ in range(2):
        b.run()
    torch.cuda.synchronize()
    st = ctx.status()
    assert st["flags"] == 0
    for i, sc in enumerate(scenes):
        ref = O.solve64(sc, O.params())
        what = f"persistent={persistent} lds_batch={lds_batch} scene {i}"
        assert_A(_A(b, i), ref["A"], ref["slack"], what=what)
        S64, m64 = O.assign64(ref["A"], [0.0, 0.3, -0.2][i])
        assert_labels(b.S[i].cpu().numpy(), S64, m64, ref["A"], _A(b, i), what=what)
    b.close()


def test_compositing_launches_are_timed_without_a_graph(ctx):
    scenes = _uneven_scenes()
    dss = [L.DeviceScene(s) for s in scenes]
    g = L.Batch(ctx, dss, L.params(), lanes=2)
    g.run()
    with pytest.raises(RuntimeError):
        g.accumulate_ms()                  # a graph batch records no per-launch events
    b = L.Batch(ctx, dss, L.params(), lanes=2, use_graph=0)
    with pytest.raises(RuntimeError):
        b.accumulate_ms()                  # nothing run yet
    b.run()
    ms, n = b.accumulate_ms()
    assert n == b.info()["n_chunks"] and 0.0 < ms < 1000.0
    torch.cuda.synchronize()
    ctx.status()
    for i in range(len(scenes)):
        assert np.allclose(_A(b, i), _A(g, i), rtol=1e-6, atol=1e-9)
    b.close()
    g.close()
