"""Pins of the oracle's point-prompt propagation (Sec. 4.1 "2D mask generation
and association", supplement "Binary Mask Association"), CPU only.

Each pin fixes a part of the rule by something other than the oracle itself:
a planted centre recovered from its own projection (back-projection and
projection, a transposed rotation or a sign error fails), a k-d tree's
neighbours (scipy), a ray of planted centres (the least-depth choice), and
the documented special cases (ties, nothing in front, k beyond n, a camera
facing away)."""
import dataclasses

import numpy as np
from scipy.spatial import cKDTree

import oracle as O
import scenegen as sg


def _with_centres(scene, centres):
    """The scene's cameras with Gaussians at the given centres."""
    c = np.asarray(centres, dtype=np.float32)
    n = c.shape[0]
    one = np.ones(n, np.float32)
    return dataclasses.replace(
        scene, mx=c[:, 0].copy(), my=c[:, 1].copy(), mz=c[:, 2].copy(), qw=one.copy(),
        qx=0 * one, qy=0 * one, qz=0 * one, sx=0.01 * one, sy=0.01 * one, sz=0.01 * one,
        op=0.5 * one, gt=np.zeros(n, np.int32))


def _project64(scene, v, X):
    R, t = scene.R[v].astype(np.float64), scene.t[v].astype(np.float64)
    x = R @ np.asarray(X, np.float64) + t
    return (scene.fx[v] * x[0] / x[2] + scene.cx[v], scene.fy[v] * x[1] / x[2] + scene.cy[v], x[2])


def _ray_point(scene, v, px, py, d):
    """World point at camera depth d on the ray of pixel (px, py), in float64."""
    R, t = scene.R[v].astype(np.float64), scene.t[v].astype(np.float64)
    c = np.array([d * (px - scene.cx[v]) / scene.fx[v], d * (py - scene.cy[v]) / scene.fy[v], d])
    return R.T @ (c - t)


def test_planted_centre_is_recovered_from_its_projection():
    base = sg.make_config("C1")
    rng = np.random.default_rng(0)
    far = rng.normal(size=(500, 3)) * 0.2 + np.array([0.0, 0.0, 0.0])
    planted = np.array([0.31, -0.22, 0.17])
    cen = np.vstack([far, planted])
    sc = _with_centres(base, cen)
    for v in (0, 3):
        u, w, z = _project64(sc, v, planted)
        ch, nn, uv, vis = O.prompt32(sc, v, [[u, w, z]], k=1)
        assert nn[0, 0] == 500 and ch[0] == 500
        # the chosen centre carried back to the reference view lands on the prompt
        assert abs(uv[0, v, 0] - u) < 1e-3 and abs(uv[0, v, 1] - w) < 1e-3
        # and into every other view where the float64 projection puts it
        for o in range(sc.n_views):
            uo, wo, zo = _project64(sc, o, planted)
            if zo > 0.2:
                assert abs(uv[0, o, 0] - uo) < 1e-2 and abs(uv[0, o, 1] - wo) < 1e-2
                inside = 0 <= uo < sc.W[o] and 0 <= wo < sc.H[o]
                assert vis[0, o] == inside


def test_nearest_match_a_kd_tree():
    base = sg.make_config("C1")
    rng = np.random.default_rng(1)
    cen = rng.normal(size=(3000, 3)) * 0.6
    sc = _with_centres(base, cen)
    tree = cKDTree(np.stack([sc.mx, sc.my, sc.mz], 1).astype(np.float64))
    for trial in range(6):
        v = int(rng.integers(sc.n_views))
        px, py, d = rng.uniform(10, 118), rng.uniform(10, 118), rng.uniform(2.0, 5.0)
        k = int(rng.integers(1, 33))
        _, nn, _, _ = O.prompt32(sc, v, [[px, py, d]], k=k)
        X = _ray_point(sc, v, np.float32(px), np.float32(py), np.float32(d))
        dist, idx = tree.query(X, k=k + 1)
        # where the float64 distances leave no near tie at the cut, the sets agree
        if dist[k] - dist[k - 1] > 1e-4 * dist[k]:
            assert set(nn[0].tolist()) == set(idx[:k].tolist())
        # and the order is by distance
        gaps = np.diff(dist[:k])
        for j in range(k - 1):
            if gaps[j] > 1e-4 * dist[j + 1]:
                assert nn[0, j] == idx[j]


def test_least_positive_reference_depth_is_chosen():
    base = sg.make_config("C1")
    v = 2
    px, py, d = 70.0, 50.0, 4.0
    # ten centres on the prompt's ray around the back-projected point, in shuffled order
    ss = np.array([0.04, -0.03, 0.02, -0.05, 0.01, 0.03, -0.01, 0.05, -0.02, 0.0])
    ray = [_ray_point(base, v, px, py, d + s) for s in ss]
    rng = np.random.default_rng(2)
    far = rng.normal(size=(200, 3)) * 0.3 + _ray_point(base, v, px, py, 20.0)
    sc = _with_centres(base, np.vstack([far, ray]))
    ch, nn, uv, _ = O.prompt32(sc, v, [[px, py, d]], k=10)
    assert set(nn[0].tolist()) == set(range(200, 210))
    assert ch[0] == 200 + int(np.argmin(ss))       # the front-most of the ten
    assert abs(uv[0, v, 0] - px) < 1e-2 and abs(uv[0, v, 1] - py) < 1e-2
    # with k = 1 only the nearest (s = 0) is a candidate
    ch1, nn1, _, _ = O.prompt32(sc, v, [[px, py, d]], k=1)
    assert nn1[0, 0] == 209 and ch1[0] == 209


def test_ties_go_to_the_smaller_index():
    base = sg.make_config("C1")
    X = _ray_point(base, 0, 64.0, 64.0, 3.0)
    behind_it = [_ray_point(base, 0, 64.0, 64.0, d) for d in (3.5, 4.0)]
    sc = _with_centres(base, [behind_it[0], X, X, behind_it[1]])
    ch, nn, _, _ = O.prompt32(sc, 0, [[64.0, 64.0, 3.0]], k=3)
    assert nn[0].tolist() == [1, 2, 0] and ch[0] == 1


def test_nothing_in_front_gives_minus_one():
    base = sg.make_config("C1")
    v = 1
    # centres only behind the reference camera: the nearest ones cannot be chosen
    behind = [_ray_point(base, v, 64.0, 64.0, -s) for s in (0.5, 1.0, 1.5)]
    sc = _with_centres(base, behind)
    ch, nn, uv, vis = O.prompt32(sc, v, [[64.0, 64.0, 1.0]], k=5)
    assert ch[0] == -1
    assert nn[0].tolist() == [0, 1, 2, -1, -1]   # k beyond n pads with -1
    assert not uv.any() and not vis.any()


def test_camera_facing_away_sees_nothing():
    base = sg.make_config("C1")
    X = _ray_point(base, 0, 64.0, 64.0, 3.0)
    sc = _with_centres(base, [X])
    R = sc.R.copy()
    t = sc.t.copy()
    # view 1 becomes view 0 turned half a turn about its own y axis
    flip = np.diag([-1.0, 1.0, -1.0]).astype(np.float32)
    R[1] = flip @ R[0]
    t[1] = flip @ t[0]
    sc = dataclasses.replace(sc, R=R, t=t)
    ch, _, uv, vis = O.prompt32(sc, 0, [[64.0, 64.0, 3.0]], k=1)
    assert ch[0] == 0 and vis[0, 0] == 1 and vis[0, 1] == 0
    assert uv[0, 1].tolist() == [0.0, 0.0]


def test_prompts_are_independent():
    base = sg.make_config("C1")
    prompts = [[30.0, 40.0, 3.5], [90.0, 80.0, 4.2], [64.0, 64.0, 4.0]]
    together = O.prompt32(base, 4, prompts, k=10)
    for p, pr in enumerate(prompts):
        alone = O.prompt32(base, 4, [pr], k=10)
        for a, b in zip(together, alone):
            assert np.array_equal(a[p], b[0])
