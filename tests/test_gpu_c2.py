"""GPU parity at the full size of the benchmark workload: 200k Gaussians
(4 clustered objects + background shell), 50 orbit views at 640x480, binary
masks with boundary erosion, background bias swept over {0, 0.2, 0.5}. The GPU
runs in the bench's launch configuration (all 50 views per call)."""
import numpy as np
import pytest
import torch

import oracle as O
import scenegen as sg
from paper_2409_08270_amd import _lib as L
from paper_2409_08270_amd.solve import Solver, tiles_of
from tests._lists import check_chunk_lists
from tests._parity import assert_A, assert_labels, log

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

SAMPLE = [0, 17, 33, 49]


@pytest.fixture(scope="module")
def c2():
    log("[c2] generating scene C2 (seed 2)")
    sc = sg.make_config("C2")
    ds = L.DeviceScene(sc)
    ctx = L.Context()
    solver = Solver(ctx, ds)
    log("[c2] batched solve, 50 views in one call")
    out = solver.solve(chunk=sc.n_views)
    torch.cuda.synchronize()
    st = ctx.status()
    return sc, ds, ctx, solver, out, st


@pytest.fixture(scope="module")
def ref(c2):
    sc = c2[0]
    log("[c2] oracle on all 50 views (float64)")
    return O.solve64(sc, O.params())


def test_graph_batch_lists_are_bit_exact_on_sampled_views(c2):
    # the tile lists the timed batched solve itself builds (packed per-view pair
    # sort, span codes, per-tile counts and ranges), chunk by chunk, on two lanes
    sc, ds, ctx, solver, out, st = c2
    b = L.Batch(ctx, [ds], solver.prm, gammas=[0.0], lanes=2)
    info = b.info()
    n, chunks, packed = check_chunk_lists(b, [sc], [(0, v) for v in SAMPLE], solver.prm, "C2 batch")
    log(f"[c2] batch lists: {n} entries compared bit for bit over views {SAMPLE}; {chunks} chunks, "
        f"{packed} packed")
    assert info["n_chunks"] >= 2 and packed >= 1
    b.close()


def test_call_bins_are_bit_exact_on_sampled_views(c2):
    sc, ds, ctx, solver, out, st = c2
    bins = solver.bins
    prm = solver.prm
    n = out["pairs"][0]
    vals = bins.vals[:n].cpu().numpy().view(np.uint32)
    ranges = bins.ranges.cpu().numpy().view(np.uint32).astype(np.int64)
    base = 0
    bases = []
    for v in range(sc.n_views):
        bases.append(base)
        base += tiles_of(int(sc.W[v]), int(sc.H[v]), prm)
    for v in SAMPLE:
        b = O.bin_view(sc, v, O.params())
        T = b["ranges"].shape[0]
        r = ranges[bases[v]:bases[v] + T]
        nonempty = r[:, 1] > r[:, 0]
        lo = r[nonempty, 0].min()
        hi = r[nonempty, 1].max()
        assert np.array_equal(vals[lo:hi], b["g"]), f"view {v}"
        on = b["ranges"][:, 1] > b["ranges"][:, 0]
        assert np.array_equal(nonempty, on)
        assert np.array_equal(r[on] - lo, b["ranges"][on].astype(np.int64))


def test_A_and_labels_match_the_oracle_at_full_size(c2, ref):
    sc, ds, ctx, solver, out, st = c2
    A = (out["A_hi"].double() + out["A_lo"].double()).cpu().numpy()
    assert_A(A, ref["A"], ref["slack"], what="C2 full")
    log(f"[c2] blends gpu {st['blends']} oracle {ref['blends']}; in-support evaluations gpu {st['evaluated']} "
        f"oracle {ref['evaluated']}")
    assert abs(st["blends"] - ref["blends"]) <= 1e-3 * ref["blends"]
    n, E = sc.n, sc.E
    for gamma in (0.0, 0.2, 0.5):
        S = torch.empty((E, n), dtype=torch.uint8, device="cuda")
        ctx.fs_assign(out["A_hi"], out["A_lo"], n, E, gamma, S, None)
        S64, m64 = O.assign64(ref["A"], gamma)
        assert_labels(S.cpu().numpy(), S64, m64, ref["A"], A, what=f"C2 gamma={gamma}")


def test_graph_batch_matches_the_oracle_at_full_size(c2, ref):
    # the launch configuration the benchmark times: the whole solve as one graph
    sc, ds, ctx, solver, out, st = c2
    b = L.Batch(ctx, [ds], solver.prm, gammas=[0.2])
    b.run()
    torch.cuda.synchronize()
    st2 = ctx.status()
    A = (b.A_hi[0].double() + b.A_lo[0].double()).cpu().numpy()
    assert_A(A, ref["A"], ref["slack"], what="C2 graph batch")
    log(f"[c2] graph batch: pairs emitted {st2['pairs_emitted']} of {b.info()['pairs']} planned")
    assert abs(st2["blends"] - ref["blends"]) <= 1e-3 * ref["blends"]
    S64, m64 = O.assign64(ref["A"], 0.2)
    assert_labels(b.S[0].cpu().numpy(), S64, m64, ref["A"], A, what="C2 graph batch gamma=0.2")


def test_batched_equals_per_view(c2):
    sc, ds, ctx, solver, out, st = c2
    per = Solver(ctx, ds).solve(chunk=1)
    torch.cuda.synchronize()
    ctx.status()
    a = (out["A_hi"].double() + out["A_lo"].double()).cpu().numpy()
    b = (per["A_hi"].double() + per["A_lo"].double()).cpu().numpy()
    d = np.abs(a - b).sum(1)
    s = np.abs(a).sum(1)
    assert d.sum() <= 1e-6 * s.sum()
    assert np.all(d <= 1e-5 * s + 1e-9)
    assert sum(per["pairs"]) == out["pairs"][0]


def test_column_sums_equal_accumulated_alpha_per_label(c2):
    # Eq. (7): column e of A = sum over pixels labelled e of (1 - T_final)
    sc, ds, ctx, solver, out, st = c2
    n, E = sc.n, sc.E
    A_hi = torch.zeros((n, E), dtype=torch.float32, device="cuda")
    A_lo = torch.zeros((n, E), dtype=torch.float32, device="cuda")
    px = sc.pixels()
    tf = torch.empty(px, dtype=torch.float32, device="cuda")
    nb = torch.empty(px, dtype=torch.int32, device="cuda")
    ctx.status()  # start the counters from zero
    solver.accumulate_views(range(sc.n_views), A_hi, A_lo, L.FS_RED_AUTO, tf, nb)
    st2 = ctx.status()
    A = (A_hi.double() + A_lo.double()).cpu().numpy()
    masks = ds.masks.cpu().numpy()
    acc = 1.0 - tf.double().cpu().numpy()
    for e in range(E):
        want = acc[masks == e].sum()
        assert abs(A[:, e].sum() - want) <= 1e-5 * want
    assert st2["blends"] == int(nb.sum().item())
