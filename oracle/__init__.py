"""CPU oracle for the FlashSplat splat-and-accumulate pass and its assignment.

TEST INFRASTRUCTURE ONLY: tests, the smoke check and the bench's CPU-baseline
leg may use it; the GPU library never does. It shares no code with the GPU
path; both sides read the same inputs from `scenegen`.

Pieces (paper sections in brackets):
  project32 / bin_view   strict binary32 projection and tile binning
                         [Sec. 3.1]; the reference of the bit-exact contract
  listed_rows32          the tile-listing definition applied to arbitrary
                         splats (mean, covariance, rectangle)
  project64              binary64 mean2D / conic [Sec. 3.1]
  composite64 / solve64  binary64 alpha compositing, A = sum of alpha*T per
                         (Gaussian, pixel label) [Eq. (1), Eq. (7), Eq. (8),
                         Listing 1 of the supplement]
  render64               Eq. (1) with an arbitrary per-Gaussian property
  weights64              dense per-pixel weights (tiny scenes only)
  render_masks64         novel-view masks: per-object alpha and depth,
                         depth-guided or argmax label [Sec. 3.4, supplement]
  assign64               L1-normalised, background-biased argmax per object
                         [Sec. 3.2 "Regularized ILP", Eq. (8), Listing 1 of the supplement]
  sweep64 / compact64    bias sweep and object extraction/removal
                         [Sec. 3.2 "Regularized ILP", Sec. 4.4]
  prompt32               point-prompt propagation: back-projection, the k
                         nearest centres, least reference depth, projection
                         into every view [Sec. 4.1, supplement "Binary Mask
                         Association"]; binary32 because its floating point
                         decides which Gaussian is chosen
  diagnose64             per-Gaussian diagnostics: objects each Gaussian
                         contributes to, subsets it falls in, overlap of each
                         subset with given labels [supplement "Scene
                         segmentation extension", Sec. 4.8 fewer masks]
  objective_eq2 / brute_force_binary   exhaustive checks of Eq. (2)/(6)
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Dict, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fs_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

# default rasterizer constants (the paper inherits them from 3DGS)
DEFAULT = dict(tile_w=16, tile_h=16, sigma_k=3.0, lowpass=0.3, znear=0.2, guard=1.3,
               alpha_min=1.0 / 255.0, alpha_max=0.99, t_min=1e-4, fp64_cond=64.0,
               band_eps=2.0 ** -10)
# no compositing thresholds besides the elliptical support
EXACT = dict(DEFAULT, alpha_min=0.0, alpha_max=1.0, t_min=0.0)

_KEYS = ["tile_w", "tile_h", "sigma_k", "lowpass", "znear", "guard",
         "alpha_min", "alpha_max", "t_min", "fp64_cond", "band_eps"]


def build(force: bool = False) -> str:
    """Compile the C oracle (strict IEEE, no FP contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
               "-ffp-contract=off", "-fno-fast-math", "-fexcess-precision=standard",
               "-o", tmp, _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        I64 = ctypes.c_int64
        I32 = ctypes.c_int32
        L.or_project32.argtypes = [I64, P, P, P, P, P, P, P, P, P]
        L.or_project32.restype = None
        L.or_bin.argtypes = [I64, P, P, P, P, P, P, P, P, I32, I32, P, P, P]
        L.or_bin.restype = I64
        L.or_project64.argtypes = [I64, P, P, P, P]
        L.or_project64.restype = None
        L.or_composite64.argtypes = [I64, P, P, P, P, P, P, P, I32, P, P, P, P, P]
        L.or_composite64.restype = None
        L.or_render64.argtypes = [I64, P, P, P, P, P, P, P, P]
        L.or_render64.restype = None
        L.or_weights64.argtypes = [I64, P, P, P, P, P, P, P]
        L.or_weights64.restype = None
        L.or_render_masks64.argtypes = [I64, P, P, P, P, P, P, P, P, I32, ctypes.c_double, I32, P, P, P]
        L.or_render_masks64.restype = None
        L.or_listed_rows32.argtypes = [I64, P, P, P, P, I32, I32, I32, I32, ctypes.c_float, I32, P]
        L.or_listed_rows32.restype = None
        _lib = L
    return _lib


def _p(a: np.ndarray):
    assert a.flags["C_CONTIGUOUS"], "arrays passed to the oracle must be C-contiguous"
    return ctypes.c_void_p(a.ctypes.data)


def params(**over) -> np.ndarray:
    d = dict(DEFAULT)
    d.update(over)
    out = np.zeros(12, np.float32)
    for i, k in enumerate(_KEYS):
        out[i] = d[k]
    return out


def _gauss(scene) -> np.ndarray:
    return np.ascontiguousarray(np.stack(scene.gaussian_arrays()).astype(np.float32))


def tiles_of(scene, v, prm) -> tuple:
    tw, th = int(prm[0]), int(prm[1])
    W, H = int(scene.W[v]), int(scene.H[v])
    return (W + tw - 1) // tw, (H + th - 1) // th


def project32(scene, v: int, prm: np.ndarray, gauss: Optional[np.ndarray] = None) -> Dict[str, np.ndarray]:
    """Strict binary32 projection of every Gaussian into view v."""
    g = _gauss(scene) if gauss is None else gauss
    n = g.shape[1]
    cam = np.ascontiguousarray(scene.camera_rows()[v])
    out = dict(flags=np.zeros(n, np.uint8), rect=np.zeros((n, 4), np.int32),
               ntiles=np.zeros(n, np.int32), depth=np.zeros(n, np.float32),
               cov=np.zeros((n, 3), np.float32), mean2d=np.zeros((n, 2), np.float32))
    lib().or_project32(n, _p(g), _p(cam), _p(prm), _p(out["flags"]), _p(out["rect"]),
                       _p(out["ntiles"]), _p(out["depth"]), _p(out["cov"]), _p(out["mean2d"]))
    return out


def listed_rows32(mean2d, cov, flags, rect, tile_w, tile_h, W, H, k=3.0, max_rows=8) -> np.ndarray:
    """Listed tiles of arbitrary splats, row by row of their tile rectangles.

    mean2d float32 [n][2], cov float32 [n][3] (a, b, c), flags uint8 [n]
    (bit 1: list the whole rectangle), rect int32 [n][4] (x0, y0, x1, y1).
    Returns int32 [n][max_rows][2]: (l, r) per tile row from y0, (-1, -1) where
    the row lists nothing or lies past y1.
    """
    mean2d = np.ascontiguousarray(mean2d, np.float32)
    cov = np.ascontiguousarray(cov, np.float32)
    flags = np.ascontiguousarray(flags, np.uint8)
    rect = np.ascontiguousarray(rect, np.int32)
    n = len(flags)
    out = np.zeros((n, max_rows, 2), np.int32)
    lib().or_listed_rows32(n, _p(mean2d), _p(cov), _p(flags), _p(rect), int(tile_w), int(tile_h),
                           int(W), int(H), float(k), int(max_rows), _p(out))
    return out


def bin_view(scene, v: int, prm: np.ndarray, proj: Optional[dict] = None) -> Dict[str, np.ndarray]:
    """Tile lists of view v in (tile, depth, id) order and per-tile [start, end)."""
    pr = project32(scene, v, prm) if proj is None else proj
    tx, ty = tiles_of(scene, v, prm)
    vis = (pr["flags"] & 1) != 0
    total = int(np.sum(pr["ntiles"][vis].astype(np.int64)))
    tile = np.zeros(max(total, 1), np.int32)
    gid = np.zeros(max(total, 1), np.uint32)
    ranges = np.zeros((tx * ty, 2), np.uint32)
    n = pr["flags"].shape[0]
    cam = np.ascontiguousarray(scene.camera_rows()[v])
    got = lib().or_bin(n, _p(pr["flags"]), _p(pr["rect"]), _p(pr["ntiles"]), _p(pr["depth"]), _p(pr["cov"]),
                       _p(pr["mean2d"]), _p(cam), _p(prm), tx, ty, _p(tile), _p(gid), _p(ranges))
    assert got == total
    return dict(tile=tile[:total], g=gid[:total], ranges=ranges, proj=pr, tiles_x=tx, tiles_y=ty)


def project64(scene, v: int, prm: np.ndarray, gauss: Optional[np.ndarray] = None) -> np.ndarray:
    g = _gauss(scene) if gauss is None else gauss
    n = g.shape[1]
    cam = np.ascontiguousarray(scene.camera_rows()[v])
    out = np.zeros((n, 5), np.float64)
    lib().or_project64(n, _p(g), _p(cam), _p(prm), _p(out))
    return out


def composite64(scene, v: int, prm: np.ndarray, bins: dict, A: np.ndarray, slack: np.ndarray,
                p64: Optional[np.ndarray] = None, want_pixels: bool = False):
    """Add view v's contributions into A (float64 [n][E]) and slack (float64 [n])."""
    if p64 is None:
        p64 = project64(scene, v, prm)
    n = scene.n
    cam = np.ascontiguousarray(scene.camera_rows()[v])
    mask = np.ascontiguousarray(scene.masks[v], dtype=np.uint8)
    W, H = int(scene.W[v]), int(scene.H[v])
    tf = np.zeros((H, W), np.float64) if want_pixels else None
    nb = np.zeros((H, W), np.int32) if want_pixels else None
    stats = np.zeros(4, np.int64)
    op = np.ascontiguousarray(scene.op)
    lst = np.ascontiguousarray(bins["g"]) if bins["g"].size else np.zeros(1, np.uint32)
    lib().or_composite64(n, _p(p64), _p(op), _p(cam), _p(prm), _p(lst), _p(bins["ranges"]),
                         _p(mask), int(scene.E), _p(A), _p(slack),
                         _p(tf) if tf is not None else None, _p(nb) if nb is not None else None, _p(stats))
    return dict(tfinal=tf, nblend=nb, blends=int(stats[0]), flagged=int(stats[1]),
                bad_labels=int(stats[2]), evaluated=int(stats[3]))


def solve64(scene, prm: Optional[np.ndarray] = None, views: Optional[Sequence[int]] = None,
            want_pixels: bool = False, E: Optional[int] = None, threads: int = 1):
    """A64 and slack over the given views (default: all), plus per-view details.

    A is a sum over views (Eq. (7)): with threads > 1 the views are split
    round-robin over that many host threads (the C routines run without the
    interpreter lock), each adding into its own A and slack, and the partial
    sums are added in thread order."""
    prm = params() if prm is None else prm
    E = scene.E if E is None else E
    views = list(range(scene.n_views) if views is None else views)
    g = _gauss(scene)

    def run(group):
        A = np.zeros((scene.n, E), np.float64)
        slack = np.zeros(scene.n, np.float64)
        per_view = {}
        tot = dict(blends=0, flagged=0, bad_labels=0, evaluated=0)
        for v in group:
            b = bin_view(scene, v, prm, project32(scene, v, prm, g))
            p64 = project64(scene, v, prm, g)
            r = composite64(scene, v, prm, b, A, slack, p64=p64, want_pixels=want_pixels)
            for k in tot:
                tot[k] += r[k]
            per_view[v] = dict(bins=b, p64=p64, **r)
        return A, slack, per_view, tot

    threads = max(1, min(int(threads), len(views)))
    if threads == 1:
        A, slack, per_view, tot = run(views)
    else:
        from concurrent.futures import ThreadPoolExecutor
        with ThreadPoolExecutor(threads) as ex:
            parts = list(ex.map(run, [views[i::threads] for i in range(threads)]))
        A, slack, per_view, tot = parts[0]
        for Ai, si, pv, ti in parts[1:]:
            A += Ai
            slack += si
            per_view.update(pv)
            for k in tot:
                tot[k] += ti[k]
    return dict(A=A, slack=slack, views=per_view, **tot)


def render64(scene, v: int, prm: np.ndarray, x: np.ndarray, bins: Optional[dict] = None,
             p64: Optional[np.ndarray] = None) -> np.ndarray:
    """Eq. (1): per-pixel sum of x_i * alpha_i * prod_{j<i}(1 - alpha_j)."""
    b = bin_view(scene, v, prm) if bins is None else bins
    p = project64(scene, v, prm) if p64 is None else p64
    cam = np.ascontiguousarray(scene.camera_rows()[v])
    W, H = int(scene.W[v]), int(scene.H[v])
    out = np.zeros((H, W), np.float64)
    xx = np.ascontiguousarray(x, dtype=np.float64)
    lst = np.ascontiguousarray(b["g"]) if b["g"].size else np.zeros(1, np.uint32)
    op = np.ascontiguousarray(scene.op)  # kept alive for the call
    lib().or_render64(scene.n, _p(p), _p(op), _p(cam), _p(prm),
                      _p(lst), _p(b["ranges"]), _p(xx), _p(out))
    return out


def depth64(scene, v: int) -> np.ndarray:
    """Camera-space depth z of every Gaussian mean in view v, binary64."""
    R = scene.R[v].astype(np.float64).reshape(3, 3)
    t = scene.t[v].astype(np.float64)
    m = np.stack([scene.mx, scene.my, scene.mz]).astype(np.float64)
    return np.ascontiguousarray(R[2] @ m + t[2])


def render_masks64(scene, v: int, prm: np.ndarray, S: np.ndarray, tau: float = 0.1, mode: int = 0,
                   bins: Optional[dict] = None, p64: Optional[np.ndarray] = None):
    """Novel-view mask of view v from per-object membership S uint8 [E][n]
    (Sec. 3.4): returns label uint8 [H][W], rho and depth float64 [E][H][W]."""
    b = bin_view(scene, v, prm) if bins is None else bins
    p = project64(scene, v, prm) if p64 is None else p64
    cam = np.ascontiguousarray(scene.camera_rows()[v])
    W, H = int(scene.W[v]), int(scene.H[v])
    S = np.ascontiguousarray(S, dtype=np.uint8)
    E = S.shape[0]
    label = np.zeros((H, W), np.uint8)
    rho = np.zeros((E, H, W), np.float64)
    depth = np.full((E, H, W), np.inf)
    lst = np.ascontiguousarray(b["g"]) if b["g"].size else np.zeros(1, np.uint32)
    op = np.ascontiguousarray(scene.op)  # arrays passed by address are kept alive for the call
    z = depth64(scene, v)
    lib().or_render_masks64(scene.n, _p(p), _p(op), _p(z), _p(cam),
                            _p(prm), _p(lst), _p(b["ranges"]), _p(S), E, float(tau), int(mode), _p(label), _p(rho),
                            _p(depth))
    return label, rho, depth


def weights64(scene, v: int, prm: np.ndarray) -> np.ndarray:
    """Dense weights alpha_i*T_i, float64 [H*W, n] (tiny scenes only)."""
    b = bin_view(scene, v, prm)
    p = project64(scene, v, prm)
    cam = np.ascontiguousarray(scene.camera_rows()[v])
    W, H = int(scene.W[v]), int(scene.H[v])
    assert W * H * scene.n <= 50_000_000
    out = np.zeros((H * W, scene.n), np.float64)
    lst = np.ascontiguousarray(b["g"]) if b["g"].size else np.zeros(1, np.uint32)
    op = np.ascontiguousarray(scene.op)  # kept alive for the call
    lib().or_weights64(scene.n, _p(p), _p(op), _p(cam), _p(prm),
                       _p(lst), _p(b["ranges"]), _p(out))
    return out


# --------------------------------------------------------------------------
# assignment

def assign64(A: np.ndarray, gamma: float = 0.0):
    """Closed-form assignment for every object t (Eq. (8), Sec. 3.2 bias).

    For row g and object t: a = A[g,t], o = sum_{e != t} A[g,e] (others);
    normalise (o, a) by max(o + a, 1e-12) (L1 normalisation as in the
    supplementary PyTorch listing, whose normalize uses eps = 1e-12); the
    Gaussian belongs to t iff a_n > o_n + gamma (ties go to "others", the
    first index of the argmax). margin = |a_n - o_n - gamma|.
    Returns S uint8 [E][n] and margin float64 [E][n].
    """
    A = np.asarray(A, dtype=np.float64)
    n, E = A.shape
    # sum over e != t via exclusive prefix + exclusive suffix sums (no subtraction)
    pre = np.zeros_like(A)
    pre[:, 1:] = np.cumsum(A[:, :-1], axis=1)
    suf = np.zeros_like(A)
    suf[:, :-1] = np.cumsum(A[:, :0:-1], axis=1)[:, ::-1]
    others = pre + suf
    s = np.maximum(A + others, 1e-12)
    a_n = A / s
    o_n = others / s
    S = (a_n > o_n + gamma).T.astype(np.uint8)
    margin = np.abs(a_n - o_n - gamma).T
    return np.ascontiguousarray(S), np.ascontiguousarray(margin)


def sweep64(A: np.ndarray, gammas: Sequence[float]):
    """Labels and member counts for several background biases (the bias of
    Sec. 3.2 "Regularized ILP for Noise Reduction", adjusted interactively once
    A is known, Sec. 4.2): the closed-form assignment evaluated per bias.
    Returns S uint8 [K][E][n] and counts int64 [K][E]."""
    S = np.stack([assign64(A, g)[0] for g in gammas])
    return S, S.sum(axis=2).astype(np.int64)


def compact64(arrays: Sequence[np.ndarray], select: np.ndarray, keep_selected: bool):
    """Object extraction (keep_selected) or removal (Sec. 4.4): the Gaussians
    whose selection flag matches, in their original order, by boolean
    indexing. Returns (kept arrays, source indices)."""
    mask = (np.asarray(select) != 0) == bool(keep_selected)
    idx = np.nonzero(mask)[0]
    return [np.asarray(a)[mask] for a in arrays], idx


def diagnose64(A: Optional[np.ndarray], S: Optional[np.ndarray] = None, gt: Optional[np.ndarray] = None,
               rel_eps: float = 0.0, E: Optional[int] = None):
    """Per-Gaussian diagnostics of a solved scene.

    contrib[c]: Gaussians with exactly c objects e where A[g][e] > rel_eps * t_g,
      t_g = sum over e of A[g][e] taken in order e = 0, 1, ... (binary64), the
      number of objects a Gaussian is shared by (supplement "Scene segmentation
      extension");
    member[m]: Gaussians held by exactly m rows of S (Sec. 3.3: more than one
      only for a negative bias);
    overlap[e] = (|S_e and gt = e|, |S_e|, |gt = e|), read as an IoU in the
      fewer-masks ablation (Sec. 4.8).
    A: float64 [n][E] or None; S: [E][n] or None; gt: int [n] or None."""
    out = [None, None, None]
    if A is not None:
        A = np.asarray(A, np.float64)
        n, E = A.shape
        t = np.zeros(n)
        for e in range(E):
            t = t + A[:, e]
        c = (A > np.float64(rel_eps) * t[:, None]).sum(axis=1)
        out[0] = np.bincount(c, minlength=E + 1).astype(np.uint64)
    if S is not None:
        S = np.asarray(S) != 0
        E = S.shape[0]
        out[1] = np.bincount(S.sum(axis=0), minlength=E + 1).astype(np.uint64)
        if gt is not None:
            gt = np.asarray(gt)
            ov = np.zeros((E, 3), np.uint64)
            for e in range(E):
                ov[e] = (np.sum(S[e] & (gt == e)), np.sum(S[e]), np.sum(gt == e))
            out[2] = ov
    return tuple(out)


def iou_of(overlap: np.ndarray) -> np.ndarray:
    """Per-object IoU from diagnose64's overlap counts (NaN where both sets are empty)."""
    ov = np.asarray(overlap, np.float64)
    union = ov[:, 1] + ov[:, 2] - ov[:, 0]
    with np.errstate(invalid="ignore", divide="ignore"):
        return np.where(union > 0, ov[:, 0] / union, np.nan)


def prompt32(scene, ref_view: int, prompts, k: int = 10, znear: float = 0.2):
    """Point-prompt propagation (Sec. 4.1 "2D mask generation and association",
    supplement "Binary Mask Association"), in binary32 with every sum in a fixed
    left-to-right order, since the distances and depths decide which Gaussian
    is chosen.

    For each prompt (px, py, d) on view ref_view (R world-to-camera, pinhole
    fx, fy, cx, cy):
      1. back-project: camera point d * ((px - cx) / fx, (py - cy) / fy, 1),
         world point R^T (camera point - t);
      2. the k centres of least squared L2 distance, ties to the smaller index
         (a stable sort of the distances);
      3. of those, the one of least positive depth in the reference view
         (ties to the smaller index), or -1;
      4. its centre projected into every view: x = R m + t, kept where
         x_z > znear; (u, v) = (fx x_x / x_z + cx, fy x_y / x_z + cy); visible
         where 0 <= u < W and 0 <= v < H.
    Returns (chosen [P], nearest [P, k] (-1 past n), uv [P, V, 2], visible [P, V])."""
    f = np.float32
    pr = np.asarray(prompts, dtype=f).reshape(-1, 3)
    P, V, n = pr.shape[0], scene.n_views, scene.n
    m = np.stack([scene.mx, scene.my, scene.mz]).astype(f)      # [3, n]
    R, t = scene.R.astype(f), scene.t.astype(f)
    chosen = np.full(P, -1, np.int64)
    nearest = np.full((P, k), -1, np.int64)
    uv = np.zeros((P, V, 2), f)
    vis = np.zeros((P, V), np.uint8)
    Rr, tr = R[ref_view], t[ref_view]
    for p in range(P):
        px, py, d = pr[p]
        # step 1
        c = np.array([d * ((px - scene.cx[ref_view]) / scene.fx[ref_view]) - tr[0],
                      d * ((py - scene.cy[ref_view]) / scene.fy[ref_view]) - tr[1],
                      d - tr[2]], dtype=f)
        X = [(Rr[0, i] * c[0] + Rr[1, i] * c[1]) + Rr[2, i] * c[2] for i in range(3)]
        # step 2
        dd = [m[i] - X[i] for i in range(3)]
        d2 = (dd[0] * dd[0] + dd[1] * dd[1]) + dd[2] * dd[2]
        order = np.argsort(d2, kind="stable")[:k]
        nearest[p, :len(order)] = order
        # step 3
        z = ((Rr[2, 0] * m[0, order] + Rr[2, 1] * m[1, order]) + Rr[2, 2] * m[2, order]) + tr[2]
        front = [(z[j], int(order[j])) for j in range(len(order)) if z[j] > 0]
        if not front:
            continue
        best = min(front)[1]
        chosen[p] = best
        # step 4
        mb = m[:, best]
        for v in range(V):
            x = [((R[v, i, 0] * mb[0] + R[v, i, 1] * mb[1]) + R[v, i, 2] * mb[2]) + t[v, i] for i in range(3)]
            if not x[2] > f(znear):
                continue
            u = scene.fx[v] * (x[0] / x[2]) + scene.cx[v]
            w = scene.fy[v] * (x[1] / x[2]) + scene.cy[v]
            uv[p, v] = (u, w)
            vis[p, v] = 1 if (u >= 0 and u < f(scene.W[v]) and w >= 0 and w < f(scene.H[v])) else 0
    return chosen, nearest, uv, vis


def objective_eq2(weights: Sequence[np.ndarray], masks: Sequence[np.ndarray], P: np.ndarray) -> float:
    """Eq. (2): sum over views and pixels of |sum_i P_i alpha_i T_i - M|."""
    tot = 0.0
    for w, m in zip(weights, masks):
        tot += float(np.sum(np.abs(w @ P.astype(np.float64) - m.reshape(-1).astype(np.float64))))
    return tot


def brute_force_binary(weights: Sequence[np.ndarray], masks: Sequence[np.ndarray]):
    """Exhaustive minimum of Eq. (2) over all P in {0,1}^n (n <= 16)."""
    n = weights[0].shape[1]
    assert n <= 16
    best, best_P, vals = None, None, np.zeros(1 << n)
    for code in range(1 << n):
        P = np.array([(code >> i) & 1 for i in range(n)], np.float64)
        f = objective_eq2(weights, masks, P)
        vals[code] = f
        if best is None or f < best:
            best, best_P = f, P
    return best, best_P, vals
