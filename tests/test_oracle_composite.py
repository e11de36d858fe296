"""Pins of the oracle's compositing and accumulation (CPU only).

Expected values come from closed forms (one or two Gaussians, with alpha from
an explicit matrix inverse), from invariants that the paper's formulation
implies (Eq. (1): the blend weights and the final transmittance telescope to
one; Lemma 1; Eq. (7): the columns of A partition the accumulated alpha by
label; A is a sum over views), and from an independent rendering of Eq. (1).
"""
import math

import numpy as np
import pytest

import oracle as O
import scenegen as sg
from tests import _pins

PRM = O.params()
EXACT = O.params(**{k: O.EXACT[k] for k in ("alpha_min", "alpha_max", "t_min")})
LP = float(PRM[3])


def _eye_pose():
    return (np.eye(3), np.zeros(3))


def test_single_gaussian_weights_are_alpha():
    sc = sg.make_custom([[0.05, -0.03, 3.0]], [[0.12, 0.06, 0.09]], [[0.9, 0.2, -0.1, 0.3]], [0.8],
                        [_eye_pose()], W=32, H=32)
    S2, mean, _ = _pins.cov2_expected(sc, 0, 0, LP)
    w = O.weights64(sc, 0, EXACT)[:, 0].reshape(32, 32)
    exp = np.array([[_pins.gaussian_alpha(S2, mean, (k + 0.5, j + 0.5), float(sc.op[0]))
                     for k in range(32)] for j in range(32)])
    assert np.allclose(w, exp, rtol=1e-6, atol=1e-12)
    # A splits the same weights by label; T_final = 1 - alpha
    mask = (np.arange(32)[None, :] >= 16).astype(np.uint8) * np.ones((32, 1), np.uint8)
    sc.masks = [mask]
    r = O.solve64(sc, EXACT, want_pixels=True)
    assert r["A"][0, 0] == pytest.approx(exp[:, :16].sum(), rel=1e-6)
    assert r["A"][0, 1] == pytest.approx(exp[:, 16:].sum(), rel=1e-6)
    assert np.allclose(r["views"][0]["tfinal"], 1.0 - exp, rtol=0, atol=1e-7)


def test_two_gaussians_front_to_back():
    # the nearer Gaussian (larger id here) occludes the farther one
    sc = sg.make_custom([[0.0, 0.0, 4.0], [0.02, 0.01, 2.5]], [[0.1, 0.1, 0.1], [0.05, 0.08, 0.06]],
                        [[1, 0, 0, 0], [0.8, 0.1, 0.5, 0.2]], [0.7, 0.6], [_eye_pose()], W=32, H=32)
    S_far, m_far, _ = _pins.cov2_expected(sc, 0, 0, LP)
    S_near, m_near, _ = _pins.cov2_expected(sc, 1, 0, LP)
    w = O.weights64(sc, 0, EXACT)
    for j in range(32):
        for k in range(32):
            a_near = _pins.gaussian_alpha(S_near, m_near, (k + 0.5, j + 0.5), float(sc.op[1]))
            a_far = _pins.gaussian_alpha(S_far, m_far, (k + 0.5, j + 0.5), float(sc.op[0]))
            assert w[j * 32 + k, 1] == pytest.approx(a_near, rel=1e-6, abs=1e-12)
            assert w[j * 32 + k, 0] == pytest.approx(a_far * (1.0 - a_near), rel=1e-6, abs=1e-12)


def test_early_termination_does_not_add_the_crossing_gaussian():
    # five identical co-centred Gaussians of peak alpha 0.95 at increasing depth:
    # T = 1, 0.05, 2.5e-3, 1.25e-4, then 6.25e-6 < t_min, so only three blend
    n = 5
    sc = sg.make_custom([[0, 0, 2.0 + 0.1 * i] for i in range(n)], [[0.3, 0.3, 0.3]] * n,
                        [[1, 0, 0, 0]] * n, [0.95] * n, [_eye_pose()], W=32, H=32)
    prm = O.params(alpha_max=0.99)
    r = O.solve64(sc, prm, want_pixels=True)
    tf = r["views"][0]["tfinal"]
    nb = r["views"][0]["nblend"]
    # pixel nearest the centre: alpha is slightly below 0.95 (pixel centre offset)
    S2, mean, _ = _pins.cov2_expected(sc, 0, 0, LP)
    j = k = 15
    a = [_pins.gaussian_alpha(*_pins.cov2_expected(sc, i, 0, LP)[:2], (k + 0.5, j + 0.5), 0.95) for i in range(n)]
    T = 1.0
    added = 0
    for ai in a:
        if T * (1 - ai) < 1e-4:
            break
        T *= (1 - ai)
        added += 1
    assert added == 3
    assert nb[j, k] == 3
    assert tf[j, k] == pytest.approx(T, rel=1e-6)
    assert tf[j, k] >= 1e-4


def test_partition_of_unity_and_all_ones_render():
    sc = sg.make_config("C1")
    for v in (0, 3):
        b = O.bin_view(sc, v, PRM)
        p64 = O.project64(sc, v, PRM)
        A = np.zeros((sc.n, sc.E))
        sl = np.zeros(sc.n)
        r = O.composite64(sc, v, PRM, b, A, sl, p64=p64, want_pixels=True)
        tf = r["tfinal"]
        # Lemma 1 / Eq. (1): sum of weights + final transmittance = 1 per pixel
        W = O.weights64(sc.subset_views([v]), 0, PRM) if sc.n * tf.size <= 50_000_000 else None
        assert np.allclose(W.sum(axis=1) + tf.reshape(-1), 1.0, rtol=0, atol=1e-12)
        assert np.all(W >= 0) and np.all(W.sum(axis=1) <= 1 + 1e-12)
        # rendering Eq. (1) with x_i = 1 reproduces the accumulated alpha
        ones = O.render64(sc, v, PRM, np.ones(sc.n), bins=b, p64=p64)
        assert np.allclose(ones, 1.0 - tf, rtol=0, atol=1e-12)
        # Eq. (7): column e of A = accumulated alpha over pixels labelled e
        for e in range(sc.E):
            assert A[:, e].sum() == pytest.approx((1.0 - tf)[sc.masks[v] == e].sum(), rel=1e-10)
        # the same weights, aggregated per Gaussian, give A
        assert np.allclose(A[:, 0] + A[:, 1], W.sum(axis=0), rtol=1e-10, atol=1e-14)


def test_view_additivity_and_label_permutation():
    sc = sg.make_config("C1")
    full = O.solve64(sc, PRM)["A"]
    a = O.solve64(sc, PRM, views=[0, 2, 4, 6])["A"]
    b = O.solve64(sc, PRM, views=[1, 3, 5, 7])["A"]
    assert np.allclose(full, a + b, rtol=1e-12, atol=1e-15)
    # relabelling the masks permutes the columns of A
    sw = sg.make_config("C1")
    sw.masks = [(1 - m).astype(np.uint8) for m in sw.masks]
    swA = O.solve64(sw, PRM)["A"]
    assert np.allclose(swA[:, ::-1], full, rtol=1e-12, atol=1e-15)


def test_eq2_equals_eq5_for_random_labellings():
    # Eq. (2) evaluated by rendering the labelling equals C + sum_i P_i (A0 - A1) (Eq. (6))
    for seed in (11, 12):
        sc = sg.make_tiny(seed, n=10, views=3, res=32, masks="raycast")
        Ws = [O.weights64(sc, v, PRM) for v in range(sc.n_views)]
        A = O.solve64(sc, PRM)["A"]
        C = sum(float(m.sum()) for m in sc.masks)
        rng = np.random.default_rng(seed)
        for _ in range(20):
            P = rng.integers(0, 2, size=sc.n).astype(np.float64)
            # render the labelling with Eq. (1) (x_i = P_i) independently of the weights
            F = 0.0
            for v in range(sc.n_views):
                Rv = O.render64(sc, v, PRM, P)
                F += float(np.abs(Rv - sc.masks[v]).sum())
            assert F == pytest.approx(C + float(P @ (A[:, 0] - A[:, 1])), rel=1e-10, abs=1e-9)
            assert F == pytest.approx(O.objective_eq2(Ws, sc.masks, P), rel=1e-10, abs=1e-9)


def test_slack_is_zero_without_thresholds_near_decisions():
    # with every threshold but the support removed and a wide support, no
    # decision is ambiguous for a lone Gaussian well inside the image
    sc = sg.make_custom([[0.0, 0.0, 3.0]], [[0.05, 0.05, 0.05]], [[1, 0, 0, 0]], [0.5],
                        [_eye_pose()], W=32, H=32)
    prm = O.params(alpha_min=0.0, alpha_max=1.0, t_min=0.0, sigma_k=7.0)
    r = O.solve64(sc, prm)
    assert r["flagged"] == 0 and r["slack"][0] == 0.0


def _inside(base, rel, sign):
    """The float32 value farthest from `base` on one side, within `rel` of it."""
    b = float(np.float32(base))
    x = np.float32(b * (1 + sign * rel))
    while abs(float(x) - b) > rel * abs(b):
        x = np.nextafter(x, np.float32(b))
    return float(x)


def _inside_k(k, rel, sign):
    """The float32 sigma_k farthest from k on one side whose k^2/2 stays within rel of k's."""
    k = float(np.float32(k))
    c = 0.5 * k * k
    x = np.float32(k * math.sqrt(1 + sign * rel))
    while abs(0.5 * float(x) * float(x) - c) > rel * c:
        x = np.nextafter(x, np.float32(k))
    return float(x)


@pytest.mark.parametrize("cfg", ["C1", "C3-small"])
def test_slack_bounds_every_threshold_flip_within_the_band(cfg):
    """The slack budget against the decisions it stands for.

    The GPU takes the three compositing decisions (support, alpha_min, t_min)
    in float32; the oracle's slack[g] bounds what deciding any of them the
    other way can change in row g, for decisions within the relative band
    band_eps of the threshold. Here the float64 oracle itself is re-run with
    each threshold moved to the edge of that band, in each direction, which
    flips exactly the decisions on that side of the band: the change of every
    row must stay within its slack. The budget must not be loose either: in
    total it stays within twice the sum of those changes, and for nearly
    every row within four times its own."""
    if cfg == "C1":
        sc, views = sg.make_config("C1"), range(8)
    else:
        sc, views = sg.make_config("C3", views=4, W=320, H=240, per_obj=6000, n_shell=20000), range(4)
    eps = float(PRM[10])
    g = O._gauss(sc)
    bins = {v: O.bin_view(sc, v, PRM, O.project32(sc, v, PRM, g)) for v in views}
    p64 = {v: O.project64(sc, v, PRM, g) for v in views}

    def solve(prm):
        A = np.zeros((sc.n, sc.E))
        sl = np.zeros(sc.n)
        for v in views:
            O.composite64(sc, v, prm, bins[v], A, sl, p64=p64[v])
        return A, sl

    A0, slack = solve(PRM)
    s = np.abs(A0).sum(axis=1)
    amin, tmin, k = float(PRM[6]), float(PRM[8]), float(PRM[2])
    moved = dict(amin_up=O.params(alpha_min=_inside(amin, eps, 1)), amin_down=O.params(alpha_min=_inside(amin, eps, -1)),
                 tmin_up=O.params(t_min=_inside(tmin, eps, 1)), tmin_down=O.params(t_min=_inside(tmin, eps, -1)),
                 support_wider=O.params(sigma_k=_inside_k(k, eps, 1)),
                 support_narrower=O.params(sigma_k=_inside_k(k, eps, -1)))
    total = np.zeros(sc.n)
    for name, prm in moved.items():
        A1, _ = solve(prm)
        d = np.abs(A1 - A0).sum(axis=1)
        assert (d > 0).sum() > 100, name  # the move does flip decisions
        over = d > slack + 1e-12 * s + 1e-15
        assert not over.any(), (name, int(over.sum()), float(np.max(d - slack)))
        total += d
    has = slack > 0
    assert slack.sum() <= 2.0 * total.sum(), (slack.sum(), total.sum())
    loose = slack > 4.0 * total + 1e-12 * s
    assert loose.sum() <= 0.03 * has.sum(), (int(loose.sum()), int(has.sum()))


def test_threaded_solve_equals_the_sequential_sum_over_views():
    # A is a sum over views (Eq. (7)): splitting the views over host threads, each
    # with its own partial A, changes only the order of the float64 additions
    sc = sg.make_config("C1", n=800, views=5, res=64)
    a = O.solve64(sc, O.params())
    b = O.solve64(sc, O.params(), threads=3)
    assert a["blends"] == b["blends"] and a["evaluated"] == b["evaluated"]
    s = np.abs(a["A"]).sum()
    assert np.abs(a["A"] - b["A"]).sum() <= 1e-13 * s
    assert np.allclose(a["slack"], b["slack"], rtol=1e-12, atol=1e-18)
    assert sorted(b["views"]) == list(range(5))
