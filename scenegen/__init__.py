"""Seeded synthetic scenes for the splat-and-accumulate path.

This module generates inputs only: Gaussian parameters, pinhole cameras and
per-view label masks. It contains none of the segmentation method's
arithmetic (no projection of covariances, no compositing, no assignment), so
that both the CPU oracle and the GPU path can read the same inputs without
sharing any of the computation under test.

Conventions (the paper leaves them open; the same ones are used everywhere):
  * Gaussians are stored as float32 structure-of-arrays with post-activation
    values: linear scales and opacity in [0, 1]; quaternions (w, x, y, z) are
    unit length.
  * Cameras map world to camera with OpenCV axes (x right, y down, z forward):
    X_cam = R @ X_world + t, pixel = (fx * x / z + cx, fy * y / z + cy), and
    pixel (row j, column k) is sampled at (k + 0.5, j + 0.5).
  * Masks are uint8 [V, H, W]; label 0 is background.

Masks are produced by analytic ray casting of the ground-truth object
ellipsoids (nearest hit wins), followed by the configured noise. This is a
stand-in for the paper's SAM-generated masks, whose datasets are not
available.
"""
from __future__ import annotations

import dataclasses
import math
import os
import multiprocessing
from typing import List, Optional

import numpy as np

__all__ = ["Scene", "make_config", "make_batch", "make_tiny", "CONFIGS",
           "look_at", "orbit_cameras", "fibonacci_cameras"]


@dataclasses.dataclass
class Scene:
    name: str
    seed: int
    # Gaussians, float32 [N] each
    mx: np.ndarray
    my: np.ndarray
    mz: np.ndarray
    qw: np.ndarray
    qx: np.ndarray
    qy: np.ndarray
    qz: np.ndarray
    sx: np.ndarray
    sy: np.ndarray
    sz: np.ndarray
    op: np.ndarray
    # cameras
    R: np.ndarray      # float32 [V, 3, 3], world -> camera
    t: np.ndarray      # float32 [V, 3]
    fx: np.ndarray     # float32 [V]
    fy: np.ndarray
    cx: np.ndarray
    cy: np.ndarray
    W: np.ndarray      # int32 [V]
    H: np.ndarray      # int32 [V]
    masks: List[np.ndarray]  # uint8 [H, W] per view
    E: int
    gamma: float
    gt: np.ndarray     # int32 [N], ground-truth object label of each Gaussian

    @property
    def n(self) -> int:
        return int(self.mx.shape[0])

    @property
    def n_views(self) -> int:
        return int(self.R.shape[0])

    def gaussian_arrays(self):
        return [self.mx, self.my, self.mz, self.qw, self.qx, self.qy, self.qz,
                self.sx, self.sy, self.sz, self.op]

    def camera_rows(self) -> np.ndarray:
        """float32 [V, 18]: R (row-major 9), t (3), fx, fy, cx, cy, W, H."""
        V = self.n_views
        out = np.zeros((V, 18), dtype=np.float32)
        out[:, 0:9] = self.R.reshape(V, 9)
        out[:, 9:12] = self.t
        out[:, 12] = self.fx
        out[:, 13] = self.fy
        out[:, 14] = self.cx
        out[:, 15] = self.cy
        out[:, 16] = self.W
        out[:, 17] = self.H
        return out

    def subset_views(self, idx) -> "Scene":
        idx = list(idx)
        return dataclasses.replace(
            self, R=self.R[idx], t=self.t[idx], fx=self.fx[idx], fy=self.fy[idx],
            cx=self.cx[idx], cy=self.cy[idx], W=self.W[idx], H=self.H[idx],
            masks=[self.masks[i] for i in idx])

    def pixels(self) -> int:
        return int(np.sum(self.W.astype(np.int64) * self.H.astype(np.int64)))


# --------------------------------------------------------------------------
# cameras

def look_at(center, target, up=(0.0, 0.0, 1.0)):
    """World->camera (R, t) for an OpenCV camera at `center` looking at `target`."""
    c = np.asarray(center, dtype=np.float64)
    f = np.asarray(target, dtype=np.float64) - c
    f /= np.linalg.norm(f)
    u = np.asarray(up, dtype=np.float64)
    if abs(float(np.dot(f, u))) > 0.999:
        u = np.array([0.0, 1.0, 0.0])
    r = np.cross(f, u)
    r /= np.linalg.norm(r)
    d = np.cross(f, r)
    R = np.stack([r, d, f])
    t = -R @ c
    return R, t


def _intrinsics(W, H, hfov_deg=60.0):
    fx = W / (2.0 * math.tan(math.radians(hfov_deg) / 2.0))
    return fx, fx, W / 2.0, H / 2.0


def _pack_cameras(poses, sizes):
    V = len(poses)
    R = np.zeros((V, 3, 3), np.float32)
    t = np.zeros((V, 3), np.float32)
    fx = np.zeros(V, np.float32)
    fy = np.zeros(V, np.float32)
    cx = np.zeros(V, np.float32)
    cy = np.zeros(V, np.float32)
    W = np.zeros(V, np.int32)
    H = np.zeros(V, np.int32)
    for i, ((Ri, ti), (w, h)) in enumerate(zip(poses, sizes)):
        R[i] = Ri
        t[i] = ti
        fx[i], fy[i], cx[i], cy[i] = _intrinsics(w, h)
        W[i] = w
        H[i] = h
    return R, t, fx, fy, cx, cy, W, H


def fibonacci_cameras(n, radius, W, H):
    golden = math.pi * (3.0 - math.sqrt(5.0))
    poses = []
    for i in range(n):
        z = 1.0 - 2.0 * (i + 0.5) / n
        r = math.sqrt(max(0.0, 1.0 - z * z))
        phi = i * golden
        c = radius * np.array([r * math.cos(phi), r * math.sin(phi), z])
        poses.append(look_at(c, (0.0, 0.0, 0.0)))
    return _pack_cameras(poses, [(W, H)] * n)


def orbit_cameras(n, radius, elev_deg, W, H, phase=0.0):
    poses = []
    el = math.radians(elev_deg)
    for i in range(n):
        az = phase + 2.0 * math.pi * i / n
        c = radius * np.array([math.cos(el) * math.cos(az), math.cos(el) * math.sin(az), math.sin(el)])
        poses.append(look_at(c, (0.0, 0.0, 0.0)))
    return _pack_cameras(poses, [(W, H)] * n)


# --------------------------------------------------------------------------
# Gaussians

def _random_rotation(rng):
    q = rng.normal(size=4)
    q /= np.linalg.norm(q)
    w, x, y, z = q
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
        [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
        [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])


def _unit_quats(rng, n):
    q = rng.normal(size=(n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    return q.astype(np.float32)


def _sigmoid(x):
    return 1.0 / (1.0 + np.exp(-x))


def _uniform_in_ellipsoid(rng, n, center, axes, rot):
    d = rng.normal(size=(n, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    r = rng.random(n) ** (1.0 / 3.0)
    local = d * r[:, None] * np.asarray(axes)[None, :]
    return local @ rot.T + np.asarray(center)[None, :]


def _shell(rng, n, rmin, rmax):
    d = rng.normal(size=(n, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    r = rng.uniform(rmin, rmax, size=n)
    return d * r[:, None], r


class _Objects:
    """Ground-truth ellipsoids used for Gaussian placement and ray-cast masks."""

    def __init__(self):
        self.centers = []
        self.axes = []
        self.rots = []

    def add(self, c, a, R):
        self.centers.append(np.asarray(c, np.float64))
        self.axes.append(np.asarray(a, np.float64))
        self.rots.append(np.asarray(R, np.float64))

    def __len__(self):
        return len(self.centers)


def _raycast_view(objs: _Objects, R, t, fx, fy, cx, cy, W, H):
    """Label of the nearest ellipsoid hit per pixel (object index + 1), 0 if none."""
    R = R.astype(np.float64)
    t = t.astype(np.float64)
    C = -R.T @ t
    label = np.zeros((H, W), np.uint8)
    depth = np.full((H, W), np.inf)
    for oi in range(len(objs)):
        c, a, Q = objs.centers[oi], objs.axes[oi], objs.rots[oi]
        # conservative screen bbox of the bounding sphere
        rad = float(a.max())
        pc = R @ c + t
        if np.linalg.norm(C - c) <= rad * 1.05 or pc[2] - rad <= 1e-3:
            k0, k1, j0, j1 = 0, W, 0, H
        else:
            zc = pc[2] - rad
            ext = rad * 1.05
            xs = [(pc[0] - ext) / zc, (pc[0] + ext) / zc, (pc[0] - ext) / (pc[2] + rad), (pc[0] + ext) / (pc[2] + rad)]
            ys = [(pc[1] - ext) / zc, (pc[1] + ext) / zc, (pc[1] - ext) / (pc[2] + rad), (pc[1] + ext) / (pc[2] + rad)]
            k0 = int(max(0, math.floor(fx * min(xs) + cx) - 1))
            k1 = int(min(W, math.ceil(fx * max(xs) + cx) + 2))
            j0 = int(max(0, math.floor(fy * min(ys) + cy) - 1))
            j1 = int(min(H, math.ceil(fy * max(ys) + cy) + 2))
            if k0 >= k1 or j0 >= j1:
                continue
        kk, jj = np.meshgrid(np.arange(k0, k1) + 0.5, np.arange(j0, j1) + 0.5)
        dc = np.stack([(kk - cx) / fx, (jj - cy) / fy, np.ones_like(kk)], axis=-1)
        dw = dc @ R  # rows: R^T d
        # ellipsoid local frame
        o = ((C - c) @ Q) / a
        dl = (dw @ Q) / a
        A = np.sum(dl * dl, axis=-1)
        B = 2.0 * (dl @ o)
        Cc = float(o @ o) - 1.0
        disc = B * B - 4.0 * A * Cc
        hit = disc >= 0.0
        sq = np.sqrt(np.where(hit, disc, 0.0))
        tn = (-B - sq) / (2.0 * A)
        tf = (-B + sq) / (2.0 * A)
        tt = np.where(tn > 0.0, tn, tf)
        hit &= tt > 0.0
        sub_d = depth[j0:j1, k0:k1]
        upd = hit & (tt < sub_d)
        sub_d[upd] = tt[upd]
        label[j0:j1, k0:k1][upd] = oi + 1
    return label


def _raycast_one(args):
    objs, R, t, fx, fy, cx, cy, W, H = args
    return _raycast_view(objs, R, t, fx, fy, cx, cy, W, H).astype(np.uint8)


def _raycast_masks(objs, cams, fg_map=None):
    """Ray-cast label masks of every view. Large jobs run on a pool of fresh
    worker processes (at most 16); each view is computed the same way wherever
    it runs, so the masks do not depend on the pool."""
    R, t, fx, fy, cx, cy, W, H = cams
    n = R.shape[0]
    jobs = [(objs, R[v], t[v], float(fx[v]), float(fy[v]), float(cx[v]), float(cy[v]), int(W[v]), int(H[v]))
            for v in range(n)]
    work = float(np.sum(W.astype(np.float64) * H)) * max(1, len(objs))
    workers = max(1, min(16, os.cpu_count() or 1, n))
    if workers > 1 and work > 2e8:
        ctx = multiprocessing.get_context("spawn")
        with ctx.Pool(workers) as pool:
            out = pool.map(_raycast_one, jobs, chunksize=max(1, n // (4 * workers)))
    else:
        out = [_raycast_one(j) for j in jobs]
    if fg_map is not None:
        out = [fg_map[m].astype(np.uint8) for m in out]
    return out


def _noise_flip(rng, masks, p):
    return [np.where(rng.random(m.shape) < p, 1 - m, m).astype(np.uint8) for m in masks]


def _noise_erode(rng, masks, p, dist=2):
    from scipy.ndimage import minimum_filter
    out = []
    for m in masks:
        er = minimum_filter(m, size=2 * dist + 1, mode="nearest")
        boundary = (m == 1) & (er == 0)
        drop = boundary & (rng.random(m.shape) < p)
        mm = m.copy()
        mm[drop] = 0
        out.append(mm)
    return out


def _noise_relabel(rng, masks, p, E):
    """Each pixel, with probability p, takes one of the other E - 1 labels uniformly."""
    out = []
    for m in masks:
        sel = np.flatnonzero(rng.random(m.shape) < p)
        shift = rng.integers(1, E, size=sel.size)
        mm = m.copy()
        flat = mm.reshape(-1)
        flat[sel] = ((flat[sel].astype(np.int64) + shift) % E).astype(np.uint8)
        out.append(mm)
    return out


def _finish(name, seed, means, scales, rng, gt, cams, masks, E, gamma, quats=None, opac=None, shuffle=True):
    n = means.shape[0]
    if quats is None:
        quats = _unit_quats(rng, n)
    if opac is None:
        opac = _sigmoid(rng.normal(size=n)).astype(np.float32)
    perm = rng.permutation(n) if shuffle else np.arange(n)
    means = means[perm].astype(np.float32)
    scales = scales[perm].astype(np.float32)
    quats = quats[perm]
    opac = opac[perm].astype(np.float32)
    gt = gt[perm].astype(np.int32)
    R, t, fx, fy, cx, cy, W, H = cams
    c = lambda a: np.ascontiguousarray(a)
    return Scene(name=name, seed=seed,
                 mx=c(means[:, 0]), my=c(means[:, 1]), mz=c(means[:, 2]),
                 qw=c(quats[:, 0]), qx=c(quats[:, 1]), qy=c(quats[:, 2]), qz=c(quats[:, 3]),
                 sx=c(scales[:, 0]), sy=c(scales[:, 1]), sz=c(scales[:, 2]), op=c(opac),
                 R=R, t=t, fx=fx, fy=fy, cx=cx, cy=cy, W=W, H=H,
                 masks=masks, E=E, gamma=gamma, gt=gt)


# --------------------------------------------------------------------------
# the configurations

def _c1(seed=1, n=2000, views=8, res=128):
    """Tiny: N(0,1)^3 means, fg = inside one ellipsoid, 2% pixel flips, E=2."""
    rng = np.random.Generator(np.random.PCG64(seed))
    means = rng.normal(size=(n, 3))
    scales = np.exp(rng.normal(-3.0, 0.5, size=(n, 3)))
    objs = _Objects()
    objs.add((0.25, 0.0, 0.0), (0.9, 0.7, 0.6), np.eye(3))
    rel = (means - np.array([0.25, 0.0, 0.0])) / np.array([0.9, 0.7, 0.6])
    gt = (np.sum(rel * rel, axis=1) <= 1.0).astype(np.int32)
    cams = fibonacci_cameras(views, 4.0, res, res)
    masks = _raycast_masks(objs, cams)
    masks = _noise_flip(rng, masks, 0.02)
    return _finish("C1", seed, means, scales, rng, gt, cams, masks, 2, 0.0)


def _clusters(rng, n_obj, per_obj, center_fn, axes_lo, axes_hi):
    objs = _Objects()
    pts, gts = [], []
    for i in range(n_obj):
        c = center_fn(i)
        a = rng.uniform(axes_lo, axes_hi, size=3)
        Q = _random_rotation(rng)
        objs.add(c, a, Q)
        pts.append(_uniform_in_ellipsoid(rng, per_obj, c, a, Q))
        gts.append(np.full(per_obj, i + 1, np.int32))
    return objs, pts, gts


def _c2(seed=2, views=50, W=640, H=480, per_obj=40000, n_shell=40000):
    """4 clusters on a ring + background shell, fg = cluster 0, boundary erosion."""
    rng = np.random.Generator(np.random.PCG64(seed))

    def ring(i):
        ang = 2.0 * math.pi * i / 4
        return (1.2 * math.cos(ang), 1.2 * math.sin(ang), 0.3 if i % 2 == 0 else -0.3)

    objs, pts, gts = _clusters(rng, 4, per_obj, ring, 0.3, 0.6)
    shell, _ = _shell(rng, n_shell, 6.0, 8.0)
    means = np.concatenate(pts + [shell])
    gt = np.concatenate(gts + [np.zeros(n_shell, np.int32)])
    gt = (gt == 1).astype(np.int32)
    scales = np.exp(rng.normal(-3.0, 0.5, size=(means.shape[0], 3)))
    cams = orbit_cameras(views, 4.0, 15.0, W, H)
    fg_map = np.array([0, 1, 0, 0, 0], np.uint8)
    masks = _raycast_masks(objs, cams, fg_map)
    masks = _noise_erode(rng, masks, 0.05)
    return _finish("C2", seed, means, scales, rng, gt, cams, masks, 2, 0.0)


def _multi(name, seed, n_obj, per_obj, n_shell, views_spec, res, relabel, ball=2.5,
           axes=(0.2, 0.6), rng=None):
    rng = rng or np.random.Generator(np.random.PCG64(seed))

    def in_ball(i):
        d = rng.normal(size=3)
        d /= np.linalg.norm(d)
        return d * ball * rng.random() ** (1.0 / 3.0)

    objs, pts, gts = _clusters(rng, n_obj, per_obj, in_ball, axes[0], axes[1])
    shell, _ = _shell(rng, n_shell, 6.0, 8.0)
    means = np.concatenate(pts + [shell])
    gt = np.concatenate(gts + [np.zeros(n_shell, np.int32)])
    scales = np.exp(rng.normal(-3.0, 0.5, size=(means.shape[0], 3)))
    W, H = res
    cams = views_spec(W, H)
    E = n_obj + 1
    masks = _raycast_masks(objs, cams)
    masks = _noise_relabel(rng, masks, relabel, E)
    return _finish(name, seed, means, scales, rng, gt, cams, masks, E, 0.0)


def _c3(seed=3, views=200, W=1008, H=756, per_obj=50000, n_shell=200000):
    """16 ellipsoids + shell, two orbit rings, 3% relabels, E=17."""

    def two_rings(W, H):
        a = orbit_cameras(views // 2, 5.0, 10.0, W, H)
        b = orbit_cameras(views - views // 2, 5.0, 35.0, W, H, phase=math.pi / (views // 2))
        return tuple(np.concatenate([x, y]) for x, y in zip(a, b))

    return _multi("C3", seed, 16, per_obj, n_shell, two_rings, (W, H), 0.03)


def _c4(seed=4, views=300, W=1297, H=840, n_obj=63, n_obj_gauss=2_000_000, n_bg=1_000_000):
    """Large unbounded scene: 63 objects + far background, 30% near-degenerate splats."""
    rng = np.random.Generator(np.random.PCG64(seed))
    per_obj = n_obj_gauss // n_obj

    def in_ball(i):
        d = rng.normal(size=3)
        d /= np.linalg.norm(d)
        return d * 2.0 * rng.random() ** (1.0 / 3.0)

    objs, pts, gts = _clusters(rng, n_obj, per_obj, in_ball, 0.15, 0.45)
    d = rng.normal(size=(n_bg, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    rad = 1.0 / rng.uniform(0.02, 0.2, size=n_bg)
    bg = d * rad[:, None]
    means = np.concatenate(pts + [bg])
    gt = np.concatenate(gts + [np.zeros(n_bg, np.int32)])
    n = means.shape[0]
    scales = np.exp(rng.normal(-3.0, 0.7, size=(n, 3)))
    scales[n - n_bg:] *= (rad / 4.0)[:, None]
    kind = rng.random(n)
    disks = kind < 0.2
    needles = (kind >= 0.2) & (kind < 0.3)
    ax = rng.integers(0, 3, size=n)
    scales[disks, ax[disks]] *= 1e-4
    keep = (ax + 1) % 3
    for j in range(3):
        sel = needles & (keep != j)
        scales[sel, j] *= 1e-4
    poses = []
    for v in range(views):
        r = rng.uniform(3.0, 6.0)
        el = math.radians(rng.uniform(-10.0, 40.0))
        az = 2.0 * math.pi * v / views
        c = r * np.array([math.cos(el) * math.cos(az), math.cos(el) * math.sin(az), math.sin(el)])
        poses.append(look_at(c, rng.normal(scale=0.2, size=3)))
    cams = _pack_cameras(poses, [(W, H)] * views)
    E = n_obj + 1
    masks = _raycast_masks(objs, cams)
    masks = _noise_relabel(rng, masks, 0.05, E)
    return _finish("C4", seed, means, scales, rng, gt, cams, masks, E, 0.0)


_RES = [(320, 240), (480, 360), (640, 480), (800, 600), (1008, 756)]


def _c5_scene(s):
    seed = 5 + s
    rng = np.random.Generator(np.random.PCG64(seed))
    n = int(round(math.exp(rng.uniform(math.log(50_000), math.log(800_000)))))
    E = int(rng.integers(2, 33))
    V = int(rng.integers(20, 121))
    W, H = _RES[int(rng.integers(0, len(_RES)))]
    n_obj = E - 1
    n_shell = max(1, n // 5)
    per_obj = max(1, (n - n_shell) // n_obj)
    n_shell = n - per_obj * n_obj

    def two_rings(W, H):
        a = orbit_cameras(V // 2, 5.0, 10.0, W, H)
        b = orbit_cameras(V - V // 2, 5.0, 35.0, W, H, phase=math.pi / max(1, V // 2))
        return tuple(np.concatenate([x, y]) for x, y in zip(a, b))

    return _multi(f"C5.{s}", seed, n_obj, per_obj, n_shell, two_rings, (W, H), 0.03, rng=rng)


def make_batch(n_scenes=32, first=0):
    """The uneven multi-scene batch: scenes 5+s for s in [first, first+n_scenes)."""
    return [_c5_scene(s) for s in range(first, first + n_scenes)]


_ARRAYS = ("mx", "my", "mz", "qw", "qx", "qy", "qz", "sx", "sy", "sz", "op", "R", "t", "fx", "fy", "cx", "cy",
           "W", "H", "gt")


def save_scenes(path: str, scenes) -> None:
    """Writes scenes to one uncompressed .npz (no pickled objects): every array,
    the masks of each scene concatenated, and the scalar fields."""
    out = {"n_scenes": np.array(len(scenes))}
    for i, sc in enumerate(scenes):
        for f in _ARRAYS:
            out[f"{i}.{f}"] = getattr(sc, f)
        out[f"{i}.masks"] = np.concatenate([m.reshape(-1) for m in sc.masks]) if sc.masks else np.zeros(0, np.uint8)
        out[f"{i}.meta"] = np.array([sc.seed, sc.E], np.int64)
        out[f"{i}.gamma"] = np.array(sc.gamma, np.float64)
        out[f"{i}.name"] = np.frombuffer(sc.name.encode(), np.uint8)
    tmp = path + ".tmp.npz"
    np.savez(tmp, **out)
    os.replace(tmp, path)


def load_scenes(path: str):
    """Scenes written by save_scenes."""
    z = np.load(path, allow_pickle=False)
    scenes = []
    for i in range(int(z["n_scenes"])):
        kw = {f: z[f"{i}.{f}"] for f in _ARRAYS}
        flat = z[f"{i}.masks"]
        masks, off = [], 0
        for w, h in zip(kw["W"], kw["H"]):
            masks.append(flat[off:off + int(w) * int(h)].reshape(int(h), int(w)))
            off += int(w) * int(h)
        seed, E = (int(x) for x in z[f"{i}.meta"])
        scenes.append(Scene(name=bytes(z[f"{i}.name"]).decode(), seed=seed, masks=masks, E=E,
                            gamma=float(z[f"{i}.gamma"]), **kw))
    return scenes


def make_batch_cached(n_scenes: int = 32, cache_dir: Optional[str] = None):
    """make_batch(n_scenes), read from (or written to) cache_dir when it is given."""
    if not cache_dir:
        return make_batch(n_scenes)
    path = os.path.join(cache_dir, f"c5_{n_scenes}.npz")
    if os.path.exists(path):
        return load_scenes(path)
    scenes = make_batch(n_scenes)
    os.makedirs(cache_dir, exist_ok=True)
    save_scenes(path, scenes)
    return scenes


def make_tiny(seed, n=10, views=3, res=32, E=2, spread=0.25, masks="random"):
    """Tiny, heavily overlapping scenes for exhaustive checks (N <= 12)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    means = rng.normal(scale=spread, size=(n, 3))
    scales = np.exp(rng.normal(-1.6, 0.3, size=(n, 3)))
    quats = _unit_quats(rng, n)
    opac = rng.uniform(0.3, 0.95, size=n).astype(np.float32)
    cams = fibonacci_cameras(views, 3.0, res, res)
    if masks == "random":
        mk = [rng.integers(0, E, size=(res, res)).astype(np.uint8) for _ in range(views)]
    else:
        objs = _Objects()
        objs.add((0.1, 0.0, 0.0), (0.3, 0.25, 0.2), np.eye(3))
        mk = _raycast_masks(objs, cams)
    gt = np.zeros(n, np.int32)
    return _finish(f"tiny{seed}", seed, means, scales, rng, gt, cams, mk, E, 0.0,
                   quats=quats, opac=opac, shuffle=False)


CONFIGS = {"C1": _c1, "C2": _c2, "C3": _c3, "C4": _c4}


def make_config(name: str, seed: Optional[int] = None, **kw) -> Scene:
    fn = CONFIGS[name]
    if seed is not None:
        kw["seed"] = seed
    return fn(**kw)


def make_custom(means, scales, quats, opacity, poses, W=32, H=32, masks=None, E=2,
                focal=None, name="custom"):
    """Scene from explicit Gaussians and (R, t) world->camera poses (tests)."""
    means = np.asarray(means, np.float32).reshape(-1, 3)
    scales = np.asarray(scales, np.float32).reshape(-1, 3)
    quats = np.asarray(quats, np.float32).reshape(-1, 4)
    n = means.shape[0]
    V = len(poses)
    R = np.stack([np.asarray(r, np.float32) for r, _ in poses])
    t = np.stack([np.asarray(tt, np.float32) for _, tt in poses])
    f = np.float32(focal if focal is not None else W / (2.0 * math.tan(math.radians(30.0))))
    if masks is None:
        masks = [np.zeros((H, W), np.uint8) for _ in range(V)]
    c = np.ascontiguousarray
    return Scene(name=name, seed=0,
                 mx=c(means[:, 0]), my=c(means[:, 1]), mz=c(means[:, 2]),
                 qw=c(quats[:, 0]), qx=c(quats[:, 1]), qy=c(quats[:, 2]), qz=c(quats[:, 3]),
                 sx=c(scales[:, 0]), sy=c(scales[:, 1]), sz=c(scales[:, 2]),
                 op=c(np.asarray(opacity, np.float32).reshape(-1)),
                 R=R, t=t, fx=np.full(V, f, np.float32), fy=np.full(V, f, np.float32),
                 cx=np.full(V, W / 2.0, np.float32), cy=np.full(V, H / 2.0, np.float32),
                 W=np.full(V, W, np.int32), H=np.full(V, H, np.int32),
                 masks=[np.asarray(m, np.uint8) for m in masks], E=E, gamma=0.0,
                 gt=np.zeros(n, np.int32))
