"""Pins of the oracle's novel-view mask renderer (Sec. 3.4), CPU only:
closed forms for one and two Gaussians, the full-scene alpha of the
compositing oracle, the depth-guided and argmax label rules, and a round trip
from ground-truth labels back to the input masks."""
import numpy as np
import pytest

import oracle as O
import scenegen as sg
from tests import _pins

LP = 0.3
EXACT = O.params(**O.EXACT)


def _eye_pose():
    return (np.eye(3), np.zeros(3))


def test_one_gaussian_per_object_closed_form():
    # two separated Gaussians, one per object: rho_e is the Gaussian's own alpha, D_e its depth
    sc = sg.make_custom([[-0.25, 0.0, 3.0], [0.3, 0.05, 4.0]], [[0.08, 0.06, 0.07], [0.09, 0.1, 0.05]],
                        [[1, 0, 0, 0], [0.9, 0.1, -0.2, 0.3]], [0.8, 0.6], [_eye_pose()], W=48, H=32, E=3)
    S = np.array([[0, 0], [1, 0], [0, 1]], np.uint8)
    lab, rho, depth = O.render_masks64(sc, 0, EXACT, S, tau=0.1, mode=0)
    for e, g in ((1, 0), (2, 1)):
        S2, mean, p = _pins.cov2_expected(sc, g, 0, LP)
        exp = np.array([[_pins.gaussian_alpha(S2, mean, (k + 0.5, j + 0.5), float(sc.op[g])) for k in range(48)]
                        for j in range(32)])
        assert np.allclose(rho[e], exp, rtol=1e-6, atol=1e-12)
        seen = exp > 0
        assert np.allclose(depth[e][seen], p[2], rtol=1e-12)
        assert np.all(np.isinf(depth[e][~seen]))
    # depth-guided label: the object whose alpha passes tau (they do not overlap here)
    want = np.where(rho[1] > 0.1, 1, np.where(rho[2] > 0.1, 2, 0))
    assert np.array_equal(lab, want)


def test_two_gaussians_of_one_object_and_occlusion_by_depth():
    # object 1: two overlapping Gaussians at depths 2.5 (near) and 4.0 (far); object 2: one at 3.2
    means = [[0.0, 0.0, 4.0], [0.02, 0.01, 2.5], [0.01, -0.01, 3.2]]
    sc = sg.make_custom(means, [[0.1, 0.1, 0.1], [0.05, 0.08, 0.06], [0.07, 0.07, 0.07]],
                        [[1, 0, 0, 0], [0.8, 0.1, 0.5, 0.2], [1, 0, 0, 0]], [0.7, 0.6, 0.9],
                        [_eye_pose()], W=32, H=32, E=3)
    S = np.array([[0, 0, 0], [1, 1, 0], [0, 0, 1]], np.uint8)
    lab, rho, depth = O.render_masks64(sc, 0, EXACT, S, tau=0.1, mode=0)
    S_far, m_far, p_far = _pins.cov2_expected(sc, 0, 0, LP)
    S_near, m_near, p_near = _pins.cov2_expected(sc, 1, 0, LP)
    S_mid, m_mid, p_mid = _pins.cov2_expected(sc, 2, 0, LP)
    for j in range(32):
        for k in range(32):
            px = (k + 0.5, j + 0.5)
            a_n = _pins.gaussian_alpha(S_near, m_near, px, float(sc.op[1]))
            a_f = _pins.gaussian_alpha(S_far, m_far, px, float(sc.op[0]))
            w_n, w_f = a_n, a_f * (1.0 - a_n)
            assert rho[1, j, k] == pytest.approx(w_n + w_f, rel=1e-6, abs=1e-12)
            if w_n + w_f > 0:
                dz = (w_n * p_near[2] + w_f * p_far[2]) / (w_n + w_f)
                assert depth[1, j, k] == pytest.approx(dz, rel=1e-6)
            a_m = _pins.gaussian_alpha(S_mid, m_mid, px, float(sc.op[2]))
            assert rho[2, j, k] == pytest.approx(a_m, rel=1e-6, abs=1e-12)
            # depth guidance: among objects whose alpha exceeds tau, the nearer one
            cands = [(depth[e, j, k], e) for e in (1, 2) if rho[e, j, k] > 0.1]
            assert lab[j, k] == (min(cands)[1] if cands else 0)
    # somewhere both objects pass tau and object 2 (depth 3.2) is behind object 1's near part
    both = (rho[1] > 0.1) & (rho[2] > 0.1)
    assert both.any() and np.any(lab[both] == 1)


def test_whole_scene_alpha_is_one_minus_final_transmittance():
    sc = sg.make_config("C1", n=600, views=2, res=64)
    prm = O.params()
    S = np.zeros((2, sc.n), np.uint8)
    S[1] = 1
    r = O.solve64(sc, prm, want_pixels=True)
    for v in range(2):
        lab, rho, _ = O.render_masks64(sc, v, prm, S, tau=0.1, mode=0)
        assert np.allclose(rho[1], 1.0 - r["views"][v]["tfinal"], atol=1e-12)
        assert np.array_equal(lab, (rho[1] > 0.1).astype(np.uint8))


def test_argmax_mode_includes_the_background():
    sc = sg.make_config("C1", n=600, views=1, res=64)
    prm = O.params()
    rng = np.random.default_rng(0)
    s1 = (rng.random(sc.n) < 0.5).astype(np.uint8)
    S = np.stack([1 - s1, s1])
    lab, rho, _ = O.render_masks64(sc, 0, prm, S, mode=1)
    assert np.array_equal(lab, (rho[1] > rho[0]).astype(np.uint8))  # first maximum on ties


def test_round_trip_from_ground_truth_labels():
    # masks rendered from the generator's ground-truth object labels reproduce the input masks
    sc = sg.make_config("C1")
    prm = O.params()
    S = np.stack([(sc.gt == 0), (sc.gt == 1)]).astype(np.uint8)
    ious = []
    for v in range(sc.n_views):
        lab, _, _ = O.render_masks64(sc, v, prm, S, tau=0.1, mode=0)
        m = sc.masks[v]
        inter = np.sum((lab == 1) & (m == 1))
        union = np.sum((lab == 1) | (m == 1))
        ious.append(inter / max(union, 1))
    assert np.mean(ious) > 0.7, ious
