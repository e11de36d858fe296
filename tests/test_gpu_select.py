"""GPU bias sweep and object extraction/removal against the oracle."""
import numpy as np
import pytest
import torch

import oracle as O
import scenegen as sg
from paper_2409_08270_amd import _lib as L
from paper_2409_08270_amd.solve import Solver
from tests._parity import assert_labels, log

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    return L.Context()


@pytest.fixture(scope="module")
def c1(ctx):
    sc = sg.make_config("C1")
    ds = L.DeviceScene(sc)
    out = Solver(ctx, ds).solve(chunk=sc.n_views)
    torch.cuda.synchronize()
    ctx.status()
    ref = O.solve64(sc, O.params())
    return sc, ds, out, ref


def test_sweep_equals_single_assignments_and_the_oracle(ctx, c1):
    sc, ds, out, ref = c1
    n, E = sc.n, sc.E
    gammas = [-0.6, -0.3, -0.1, 0.0, 0.05, 0.2, 0.5, 0.9]
    S = torch.empty((len(gammas), E, n), dtype=torch.uint8, device="cuda")
    counts = ctx.fs_assign_sweep(out["A_hi"], out["A_lo"], n, E, gammas, S)
    Sg = S.cpu().numpy()
    assert np.array_equal(counts, Sg.sum(axis=2))
    S64, c64 = O.sweep64(ref["A"], gammas)
    for k, g in enumerate(gammas):
        one = torch.empty((E, n), dtype=torch.uint8, device="cuda")
        ctx.fs_assign(out["A_hi"], out["A_lo"], n, E, g, one, None)
        assert np.array_equal(one.cpu().numpy(), Sg[k])  # same arithmetic as the single call
        _, m64 = O.assign64(ref["A"], g)
        Ag = (out["A_hi"].double() + out["A_lo"].double()).cpu().numpy()
        assert_labels(Sg[k], S64[k], m64, ref["A"], Ag, what=f"sweep gamma={g}")
    assert np.all(np.diff(counts, axis=0) <= 0)
    ctx.status()


def test_sweep_many_classes_and_limits(ctx):
    rng = np.random.default_rng(4)
    n, E = 5000, 64
    A = rng.gamma(0.3, 1.0, size=(n, E)).astype(np.float32)
    A[rng.random((n, E)) < 0.5] = 0
    A_hi = torch.from_numpy(A).cuda()
    gammas = list(np.linspace(-0.9, 0.9, 64))
    counts = ctx.fs_assign_sweep(A_hi, None, n, E, gammas, None)
    _, c64 = O.sweep64(A.astype(np.float64), gammas)
    # counts may differ only through entries whose margin is below 1e-4
    for k, g in enumerate(gammas):
        _, m = O.assign64(A.astype(np.float64), g)
        amb = (m < 1e-4).sum(axis=1)
        assert np.all(np.abs(counts[k] - c64[k]) <= amb)
    with pytest.raises(L.FlashSplatError):
        ctx.fs_assign_sweep(A_hi, None, n, E, list(np.zeros(65)), None)   # 4096 / 64 = 64 biases at most
    with pytest.raises(L.FlashSplatError):
        ctx.fs_assign_sweep(A_hi, None, n, E, [1.5], None)


@pytest.mark.parametrize("E", [17, 100])
def test_sweep_counts_when_waves_straddle_objects(ctx, E):
    """Row blocks that are not whole waves per object (E = 100: 40 rows, every
    wave holds two objects) and a partial last block: the counts equal the
    labels' sums, the labels equal single assignments, with or without counts."""
    rng = np.random.default_rng(E)
    n = 3001
    A = rng.gamma(0.3, 1.0, size=(n, E)).astype(np.float32)
    A[rng.random((n, E)) < 0.6] = 0
    A_hi = torch.from_numpy(A).cuda()
    gammas = [-0.4, -0.1, 0.0, 0.1, 0.3]
    S = torch.empty((len(gammas), E, n), dtype=torch.uint8, device="cuda")
    counts = ctx.fs_assign_sweep(A_hi, None, n, E, gammas, S)
    Sg = S.cpu().numpy()
    assert np.array_equal(counts, Sg.sum(axis=2))
    S2 = torch.full((len(gammas), E, n), 7, dtype=torch.uint8, device="cuda")
    assert ctx.fs_assign_sweep(A_hi, None, n, E, gammas, S2, want_counts=False) is None
    assert np.array_equal(S2.cpu().numpy(), Sg)
    for k, g in enumerate(gammas):
        one = torch.empty((E, n), dtype=torch.uint8, device="cuda")
        ctx.fs_assign(A_hi, None, n, E, g, one, None)
        assert np.array_equal(one.cpu().numpy(), Sg[k])
    ctx.status()


def test_extraction_and_removal(ctx, c1):
    sc, ds, out, ref = c1
    S = out["S"]
    sel = S[1].contiguous()  # the foreground object's Gaussians
    arrays = [a.cpu().numpy() for a in ds.arrays]
    s_np = sel.cpu().numpy()
    for keep in (True, False):
        got, idx = ctx.fs_compact(ds, sel, keep)
        want, widx = O.compact64(arrays, s_np, keep)
        assert np.array_equal(idx.cpu().numpy(), widx)
        for g, w in zip(got, want):
            assert np.array_equal(g.cpu().numpy(), w)  # a copy: bit-exact
        log(f"[compact] keep_selected={keep}: {len(widx)} of {sc.n}")
    # too small an output is reported with the size needed
    k = int(s_np.sum())
    if k > 1:
        with pytest.raises(L.FlashSplatError):
            ctx.fs_compact(ds, sel, True, capacity=k - 1)
    # empty selection
    none = torch.zeros_like(sel)
    got, idx = ctx.fs_compact(ds, none, True)
    assert idx.numel() == 0
