"""Pins of the oracle's projection and binning (CPU only).

Each expected value comes from mathematics independent of the oracle's own
formulas: closed forms for special Gaussians, a finite-difference Jacobian
with scipy's quaternion rotation for general ones, numpy's eigensolver for
the bounding radius, brute force for the tile rectangles and numpy's lexsort
for the order (paper Sec. 3.1: projection to 2D Gaussians, 16x16 tiles,
blending in depth order).
"""
import math

import numpy as np
import pytest

import oracle as O
import scenegen as sg
from tests import _pins

PRM = O.params()
LP = float(PRM[3])


def _cov_from_conic(c):
    C = np.array([[c[2], c[3]], [c[3], c[4]]])
    return np.linalg.inv(C)


def _eye_pose():
    return (np.eye(3), np.zeros(3))


def test_isotropic_on_axis_closed_form():
    # isotropic Gaussian on the optical axis: Sigma2 = (f s / z)^2 I + lowpass I
    z, s, W = 5.0, 0.1, 64
    sc = sg.make_custom([[0, 0, z]], [[s, s, s]], [[1, 0, 0, 0]], [0.5], [_eye_pose()], W=W, H=W)
    f = float(sc.fx[0])
    s = float(sc.sx[0])
    p64 = O.project64(sc, 0, PRM)[0]
    expect = (f * s / z) ** 2 + LP
    S2 = _cov_from_conic(p64)
    assert np.allclose(S2, expect * np.eye(2), rtol=1e-12, atol=1e-12)
    assert p64[0] == pytest.approx(W / 2) and p64[1] == pytest.approx(W / 2)
    pr = O.project32(sc, 0, PRM)
    assert pr["flags"][0] & 1
    assert np.allclose(pr["cov"][0], [expect, 0.0, expect], rtol=1e-6)
    r = math.ceil(3.0 * math.sqrt(expect))
    kmin = max(0, math.ceil(W / 2 - r - 0.5))
    kmax = min(W - 1, math.floor(W / 2 + r - 0.5))
    assert list(pr["rect"][0]) == [kmin // 16, kmin // 16, kmax // 16, kmax // 16]


def test_axis_aligned_anisotropic_closed_form():
    z = 4.0
    s = np.array([0.2, 0.05, 0.3])
    sc = sg.make_custom([[0, 0, z]], [s], [[1, 0, 0, 0]], [0.5], [_eye_pose()], W=64, H=48)
    f = float(sc.fx[0])
    s = np.array([sc.sx[0], sc.sy[0], sc.sz[0]], np.float64)
    S2 = _cov_from_conic(O.project64(sc, 0, PRM)[0])
    expect = np.diag([(f * s[0] / z) ** 2 + LP, (f * s[1] / z) ** 2 + LP])
    assert np.allclose(S2, expect, rtol=1e-12, atol=1e-12)


def test_general_gaussians_match_fd_jacobian():
    # random rotations, off-axis positions, several cameras
    sc = sg.make_tiny(7, n=12, views=4, res=64)
    for v in range(sc.n_views):
        p64 = O.project64(sc, v, PRM)
        pr = O.project32(sc, v, PRM)
        for g in range(sc.n):
            S2, mean, p = _pins.cov2_expected(sc, g, v, LP)
            # keep to Gaussians inside the guard band (no clamp in effect)
            lim = 1.3 * 0.5 * float(sc.W[v]) / float(sc.fx[v])
            if abs(p[0] / p[2]) > lim or abs(p[1] / p[2]) > lim or p[2] <= 0.2:
                continue
            assert np.allclose(_cov_from_conic(p64[g]), S2, rtol=2e-6, atol=1e-9)
            assert np.allclose(p64[g][:2], mean, rtol=0, atol=1e-9)
            # the binary32 covariance agrees to float32 accuracy
            assert np.allclose(pr["cov"][g], [S2[0, 0], S2[0, 1], S2[1, 1]], rtol=2e-5, atol=2e-5 * S2.max())
            assert pr["depth"][g] == pytest.approx(p[2], rel=1e-6)


def test_guard_band_clamp_freezes_jacobian():
    # beyond the guard band the Jacobian is evaluated at the clamped ray, so the
    # 2D covariance stops changing as the Gaussian moves further sideways
    z = 3.0
    lim = 1.3 * 0.5 * 64 / float(sg.make_custom([[0, 0, 1]], [[1, 1, 1]], [[1, 0, 0, 0]], [1], [_eye_pose()], W=64, H=64).fx[0])
    xs = [lim * z * 1.2, lim * z * 1.5, lim * z * 2.5]
    sc = sg.make_custom([[x, 0.3, z] for x in xs], [[0.1, 0.2, 0.15]] * 3,
                        [[0.9, 0.1, -0.3, 0.2]] * 3, [0.5] * 3, [_eye_pose()], W=64, H=64)
    S = [_cov_from_conic(c) for c in O.project64(sc, 0, PRM)]
    assert np.allclose(S[0], S[1], rtol=1e-12) and np.allclose(S[0], S[2], rtol=1e-12)
    # and inside the band it does change
    sc2 = sg.make_custom([[0.1 * z, 0.3, z], [0.3 * z, 0.3, z]], [[0.1, 0.2, 0.15]] * 2,
                         [[0.9, 0.1, -0.3, 0.2]] * 2, [0.5] * 2, [_eye_pose()], W=64, H=64)
    S2 = [_cov_from_conic(c) for c in O.project64(sc2, 0, PRM)]
    assert not np.allclose(S2[0], S2[1], rtol=1e-3)


def test_rect_is_the_support_bounding_box_by_brute_force():
    # tile rectangle = tiles holding a pixel centre within u +- ceil(3 sqrt(a)), v +- ceil(3 sqrt(c))
    sc = sg.make_tiny(3, n=12, views=3, res=48, spread=0.6)
    for v in range(sc.n_views):
        pr = O.project32(sc, v, PRM)
        W, H = int(sc.W[v]), int(sc.H[v])
        for g in range(sc.n):
            if not (pr["flags"][g] & 1):
                continue
            a, b, c = [np.float32(x) for x in pr["cov"][g]]
            rx = float(np.ceil(np.float32(3.0) * np.sqrt(a)))
            ry = float(np.ceil(np.float32(3.0) * np.sqrt(c)))
            # the box holds the whole k-sigma ellipse: its x half-extent is 3 sqrt(a) (eigen form)
            lam = np.linalg.eigvalsh(np.array([[a, b], [b, c]], np.float64))
            assert 3.0 * math.sqrt(lam[-1]) >= 3.0 * math.sqrt(float(a)) - 1e-6
            u, vv = [float(x) for x in pr["mean2d"][g]]
            tiles = set()
            for j in range(H):
                for k in range(W):
                    if abs(k + 0.5 - u) <= rx and abs(j + 0.5 - vv) <= ry:
                        tiles.add((k // 16, j // 16))
            x0, y0, x1, y1 = pr["rect"][g]
            got = {(tx, ty) for ty in range(y0, y1 + 1) for tx in range(x0, x1 + 1)} if tiles else set()
            assert got == tiles, (v, g)


def _pairs_by_tile(b):
    out = {}
    for t, g in zip(b["tile"], b["g"]):
        out.setdefault(int(g), set()).add(int(t))
    return out


@pytest.mark.parametrize("cfg", ["tiny", "C1"])
def test_tile_lists_lose_no_support_pixel_and_are_tight(cfg):
    sc = sg.make_tiny(4, n=12, views=3, res=64, spread=0.5) if cfg == "tiny" else sg.make_config("C1")
    for v in range(min(3, sc.n_views)):
        b = O.bin_view(sc, v, PRM)
        p64 = O.project64(sc, v, PRM)
        pr = b["proj"]
        tx = b["tiles_x"]
        W, H = int(sc.W[v]), int(sc.H[v])
        listed = _pairs_by_tile(b)
        jj, kk = np.mgrid[0:H, 0:W]
        for g in np.nonzero((pr["flags"] & 1) != 0)[0]:
            u, vv, A, B, C = p64[g]
            dx = kk + 0.5 - u
            dy = jj + 0.5 - vv
            q = A * dx * dx + 2 * B * dx * dy + C * dy * dy
            need = {int((j // 16) * tx + (k // 16)) for j, k in zip(*np.nonzero(q <= 9.0))}
            have = listed.get(int(g), set())
            # no pixel centre inside the support ellipse is lost
            assert need <= have, (v, g)
            if pr["flags"][g] & 2:
                continue
            # every listed tile comes close: a dense sample of its pixel-centre box reaches q <= 9 (1 + 1%)
            for t in have:
                ty_, tx_ = divmod(t, tx)
                xs = np.linspace(tx_ * 16 + 0.5, min(tx_ * 16 + 15, W - 1) + 0.5, 61) - u
                ys = np.linspace(ty_ * 16 + 0.5, min(ty_ * 16 + 15, H - 1) + 0.5, 61) - vv
                X, Y = np.meshgrid(xs, ys)
                qmin = (A * X * X + 2 * B * X * Y + C * Y * Y).min()
                assert qmin <= 9.0 * 1.01, (v, g, t, qmin)
            # each tile row's listed span is contiguous and its end tiles hold a pixel centre
            # inside 9 (1 + 2^-7), up to float32 rounding (the listing definition)
            qpix = q <= 9.0 * 1.0078125 * (1 + 1e-4)
            rows = {}
            for t in have:
                rows.setdefault(t // tx, []).append(t % tx)
            for ty_, cols in rows.items():
                assert sorted(cols) == list(range(min(cols), max(cols) + 1)), (v, g, ty_)
                for tx_ in (min(cols), max(cols)):
                    assert qpix[ty_ * 16:ty_ * 16 + 16, tx_ * 16:tx_ * 16 + 16].any(), (v, g, ty_, tx_)
            assert pr["ntiles"][g] == len(have)


def test_culling_and_visibility():
    bad = [
        ([0, 0, 3], [0.1, 0.1, 0.1], [0, 0, 0, 0], 0.5),          # zero quaternion
        ([0, 0, 3], [0.1, 0.0, 0.1], [1, 0, 0, 0], 0.5),          # zero scale
        ([0, 0, 3], [0.1, -0.1, 0.1], [1, 0, 0, 0], 0.5),         # negative scale
        ([0, float("nan"), 3], [0.1, 0.1, 0.1], [1, 0, 0, 0], 0.5),
        ([0, 0, 3], [0.1, float("inf"), 0.1], [1, 0, 0, 0], 0.5),
        ([0, 0, 3], [0.1, 0.1, 0.1], [1, 0, 0, 0], float("nan")),
        ([0, 0, 0.1], [0.1, 0.1, 0.1], [1, 0, 0, 0], 0.5),        # in front of znear
        ([0, 0, -3], [0.1, 0.1, 0.1], [1, 0, 0, 0], 0.5),         # behind the camera
        ([50, 0, 3], [0.1, 0.1, 0.1], [1, 0, 0, 0], 0.5),         # far off screen: no tiles
        ([0, 0, 3], [0.1, 0.1, 0.1], [2, 0, 0, 0], 0.5),          # unnormalised quaternion: fine
    ]
    sc = sg.make_custom([b[0] for b in bad], [b[1] for b in bad], [b[2] for b in bad],
                        [b[3] for b in bad], [_eye_pose()], W=32, H=32)
    pr = O.project32(sc, 0, PRM)
    assert list(pr["flags"][:6]) == [4] * 6
    assert pr["flags"][6] == 0 and pr["flags"][7] == 0
    assert pr["flags"][8] & 1 and pr["ntiles"][8] == 0
    assert pr["flags"][9] & 1 and pr["ntiles"][9] > 0
    # unnormalised quaternion gives the same covariance as the normalised one
    sc1 = sg.make_custom([[0, 0, 3]] * 2, [[0.1, 0.2, 0.3]] * 2, [[2, 1, 0, 0.5], [0.8, 0.4, 0, 0.2]],
                         [0.5, 0.5], [_eye_pose()], W=32, H=32)
    p = O.project64(sc1, 0, PRM)
    assert np.allclose(p[0], p[1], rtol=1e-12)


def test_fp64_predicate_flags_needles():
    # a needle (two tiny axes) projected along a diagonal is near-degenerate
    q = [math.cos(0.3), 0.0, 0.0, math.sin(0.3)]
    sc = sg.make_custom([[0, 0, 3], [0.2, 0, 3]], [[2.0, 1e-5, 1e-5], [0.1, 0.1, 0.1]],
                        [q, [1, 0, 0, 0]], [0.5, 0.5], [_eye_pose()], W=64, H=64)
    pr = O.project32(sc, 0, PRM)
    assert pr["flags"][0] & 2
    assert not (pr["flags"][1] & 2)
    # Cauchy-Binet determinant: the binary64 conic is still the inverse covariance
    S2, _, _ = _pins.cov2_expected(sc, 0, 0, LP)
    assert np.allclose(_cov_from_conic(O.project64(sc, 0, PRM)[0]), S2, rtol=1e-6)


def test_bin_order_matches_lexsort():
    sc = sg.make_config("C1")
    for v in (0, 5):
        b = O.bin_view(sc, v, PRM)
        pr = b["proj"]
        tiles = b["tile"].astype(np.int64)
        gid = b["g"].astype(np.int64)
        depth = pr["depth"][gid]
        # the pairs re-sorted by (tile, depth, id) with numpy come out unchanged
        order = np.lexsort((gid, depth, tiles))
        assert np.array_equal(order, np.arange(order.size))
        # every visible Gaussian appears exactly ntiles times
        cnt = np.bincount(gid, minlength=sc.n)
        assert np.array_equal(cnt, np.where((pr["flags"] & 1) != 0, pr["ntiles"], 0))
        T = b["ranges"].shape[0]
        st = np.searchsorted(tiles, np.arange(T), side="left")
        en = np.searchsorted(tiles, np.arange(T), side="right")
        nonempty = en > st
        assert np.array_equal(b["ranges"][nonempty, 0], st[nonempty])
        assert np.array_equal(b["ranges"][nonempty, 1], en[nonempty])
        assert np.all(b["ranges"][~nonempty] == 0)
