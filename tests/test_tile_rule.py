"""The kernels' tile-listing rule against the oracle's pixel-by-pixel definition.

The GPU binning finds each tile row's listed span from closed-form bounds of a
slightly widened ellipse plus direct tests of the centres near its boundary
(`csrc/fs_tiles.h`). The oracle applies the definition itself: every centre of
the tile row is tested (Sec. 3.1: tiles share the Gaussians whose support
reaches them). The header's functions are host-callable, so this test builds
them for the CPU and compares the two listings, bit for bit, on random splats
of every size, aspect and orientation, on means aligned with the pixel grid,
and on badly conditioned splats forced onto the float32 path (which take the
exhaustive fallback). No GPU is used.
"""
import ctypes
import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest

import oracle as O

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "native", "tile_rule_host.hip")
INC = os.path.join(ROOT, "paper_2409_08270_amd", "csrc")


def _hipcc():
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    return None


@pytest.fixture(scope="module")
def rule():
    hipcc = _hipcc()
    if hipcc is None:
        pytest.skip("hipcc not found: the host build of the tile rule needs it")
    d = tempfile.mkdtemp(prefix="fs_tile_rule_")
    so = os.path.join(d, "libtilerule.so")
    subprocess.check_call([hipcc, "-x", "hip", "--offload-arch=gfx950", "-O2", "-fPIC", "-shared", "-std=c++17",
                           "-ffp-contract=off", "-I", INC, "-o", so, SRC])
    L = ctypes.CDLL(so)
    P = ctypes.c_void_p
    I32 = ctypes.c_int32
    L.tr_row_spans.argtypes = [ctypes.c_int64, P, P, P, P, I32, I32, I32, I32, ctypes.c_float, I32, P]
    L.tr_row_spans.restype = None

    def spans(mean2d, cov, flags, rect, tw, th, W, H, max_rows):
        n = len(flags)
        out = np.zeros((n, max_rows, 2), np.int32)
        a = [np.ascontiguousarray(x) for x in (mean2d, cov, flags, rect)]
        L.tr_row_spans(n, *[P(x.ctypes.data) for x in a], tw, th, W, H, 3.0, max_rows, P(out.ctypes.data))
        return out

    yield spans
    shutil.rmtree(d, ignore_errors=True)


def _splats(rng, n, W, H, tw, th, smax, cond=64.0, force_float32=False, aligned=False):
    """Random 2D splats with the projection's rectangle and conditioning flag."""
    if aligned:
        u = (rng.integers(-40, W * 8 + 40, n) / 8.0).astype(np.float32)
        v = (rng.integers(-40, H * 8 + 40, n) / 8.0).astype(np.float32)
        s = rng.choice(np.array([0.5, 1, 1.5, 2, 3, 4, 5.5, 8, 16, 33.3], np.float32), (n, 2))
        kind = rng.integers(0, 3, n)  # axis-aligned, +45 degrees, -45 degrees
        a = np.where(kind == 0, s[:, 0] ** 2, (s[:, 0] ** 2 + s[:, 1] ** 2) / 2).astype(np.float32)
        c = np.where(kind == 0, s[:, 1] ** 2, (s[:, 0] ** 2 + s[:, 1] ** 2) / 2).astype(np.float32)
        b = np.where(kind == 0, 0, np.where(kind == 1, 1, -1) * (s[:, 0] ** 2 - s[:, 1] ** 2) / 2).astype(np.float32)
    else:
        u = rng.uniform(-30, W + 30, n).astype(np.float32)
        v = rng.uniform(-30, H + 30, n).astype(np.float32)
        ang = rng.uniform(0, np.pi, n)
        s1 = np.exp(rng.uniform(np.log(0.3), np.log(smax), n))
        s2 = np.exp(rng.uniform(np.log(0.3), np.log(smax), n))
        co, si = np.cos(ang), np.sin(ang)
        a = (co * co * s1 * s1 + si * si * s2 * s2 + 0.3).astype(np.float32)
        b = (co * si * (s1 * s1 - s2 * s2)).astype(np.float32)
        c = (si * si * s1 * s1 + co * co * s2 * s2 + 0.3).astype(np.float32)
    det = (a * c - b * b).astype(np.float32)
    deg = ~(det > 0) | ((a * c).astype(np.float32) >= np.float32(cond) * det)
    flags = np.where(deg & ~force_float32, 3, 1).astype(np.uint8)
    rx = np.ceil(np.float32(3) * np.sqrt(a))
    ry = np.ceil(np.float32(3) * np.sqrt(c))
    fk0, fk1 = np.ceil((u - rx) - np.float32(0.5)), np.floor((u + rx) - np.float32(0.5))
    fj0, fj1 = np.ceil((v - ry) - np.float32(0.5)), np.floor((v + ry) - np.float32(0.5))
    ok = ~((fk1 < 0) | (fk0 > W - 1) | (fj1 < 0) | (fj0 > H - 1) | (fk0 > fk1) | (fj0 > fj1))
    k0, k1 = np.maximum(fk0, 0).astype(np.int64), np.minimum(fk1, W - 1).astype(np.int64)
    j0, j1 = np.maximum(fj0, 0).astype(np.int64), np.minimum(fj1, H - 1).astype(np.int64)
    rect = np.stack([k0 // tw, j0 // th, k1 // tw, j1 // th], 1).astype(np.int32)
    return np.stack([u, v], 1)[ok], np.stack([a, b, c], 1)[ok], flags[ok], rect[ok]


CASES = [
    # W, H, tile, largest sigma (px), conditioning bound, float32 path forced, grid-aligned means
    (640, 480, 16, 16, 20.0, 64.0, False, False),
    (1297, 840, 16, 16, 400.0, 64.0, False, False),
    (200, 150, 32, 8, 60.0, 64.0, False, False),
    (300, 200, 12, 10, 60.0, 64.0, False, False),
    (640, 480, 16, 16, 2000.0, 64.0, False, False),
    (400, 300, 16, 16, 200.0, 1e5, True, False),
    (640, 480, 16, 16, 0.0, 64.0, False, True),
    (300, 200, 12, 10, 0.0, 64.0, False, True),
]


@pytest.mark.parametrize("case", CASES)
def test_kernel_rule_equals_pixel_definition(rule, case):
    W, H, tw, th, smax, cond, force, aligned = case
    rng = np.random.default_rng(7 + CASES.index(case))
    m, cv, f, r = _splats(rng, 40000, W, H, tw, th, smax, cond, force, aligned)
    rows = int((r[:, 3] - r[:, 1]).max()) + 1
    got = rule(m, cv, f, r, tw, th, W, H, rows)
    ref = O.listed_rows32(m, cv, f, r, tw, th, W, H, max_rows=rows)
    bad = np.nonzero((got != ref).any(axis=(1, 2)))[0]
    assert len(bad) == 0, (len(bad), m[bad[0]], cv[bad[0]], f[bad[0]], r[bad[0]])
    # the case exercises listing: most splats list something, some rows list nothing
    assert (ref[:, :, 0] >= 0).any(axis=1).mean() > 0.5
    assert ((ref[:, :, 0] < 0) & (np.arange(rows)[None, :] <= (r[:, 3] - r[:, 1])[:, None])).any()
