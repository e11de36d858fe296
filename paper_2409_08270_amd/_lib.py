"""ctypes binding of libflashsplat.so (include/flashsplat.h).

Argument marshalling only: every step of the path runs in the library's HIP
kernels. PyTorch provides device memory and the stream. The binding refuses
to run when the library is missing; there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libflashsplat.so")

FS_OK = 0
FS_ERR_ARG = -1
FS_ERR_ALLOC = -2
FS_ERR_HIP = -3
FS_ERR_CAPACITY = -4
FS_ERR_DEVICE = -5
FS_ERR_STATE = -6

FS_DEV_BAD_LABEL = 1
FS_DEV_PAIR_OVERFLOW = 2
FS_DEV_INVALID_GAUSS = 4
FS_DEV_MANY_LABELS = 8

FS_RED_AUTO = 0
FS_RED_PLAIN = 1
FS_RED_LDS = 2
FS_RED_LDS2SUM = 3
FS_RED_DET = 4

FS_NOALLOC_MAX_VIEWS = 4096
FS_NOALLOC_MAX_TILES = 1048576

FS_MASK_DEPTH = 0
FS_MASK_ARGMAX = 1

_P = ctypes.c_void_p
_F = ctypes.c_float
_I32 = ctypes.c_int32
_I64 = ctypes.c_int64


class FsGaussians(ctypes.Structure):
    _fields_ = [(k, _P) for k in ("mx", "my", "mz", "qw", "qx", "qy", "qz", "sx", "sy", "sz", "opacity")] + [("n", _I64)]


class FsCamera(ctypes.Structure):
    _fields_ = [("R", _F * 9), ("t", _F * 3), ("fx", _F), ("fy", _F), ("cx", _F), ("cy", _F),
                ("width", _I32), ("height", _I32)]


class FsParams(ctypes.Structure):
    _fields_ = [("tile_w", _I32), ("tile_h", _I32), ("sigma_k", _F), ("lowpass", _F), ("znear", _F),
                ("guard", _F), ("alpha_min", _F), ("alpha_max", _F), ("t_min", _F), ("fp64_cond", _F),
                ("fp64_conic", _I32), ("tile_order", _I32), ("count_ops", _I32), ("persistent", _I32),
                ("lds_batch", _I32)]


class FsProj(ctypes.Structure):
    _fields_ = [("rec", _P), ("rect", _P), ("ntiles", _P), ("flags", _P), ("n", _I64), ("n_views", _I32)]


class FsBins(ctypes.Structure):
    _fields_ = [("vals", _P), ("tiles", _P), ("ranges", _P), ("capacity", _I64)]


class FsPixelOut(ctypes.Structure):
    _fields_ = [("t_final", _P), ("n_blend", _P)]


class FsStatus(ctypes.Structure):
    _fields_ = [("flags", ctypes.c_uint32), ("bad_labels", _I64), ("invalid_gauss", _I64),
                ("fp64_splats", _I64), ("pairs_dropped", _I64), ("blends", _I64), ("evaluated", _I64), ("wave_steps", _I64),
                ("wave_steps_max", _I64), ("unseen", _I64),
                ("multi_member", _I64), ("low_margin", _I64), ("pairs_emitted", _I64), ("entries_staged", _I64)]

    def as_dict(self):
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


class FsScene(ctypes.Structure):
    _fields_ = [("gauss", FsGaussians), ("cams", ctypes.POINTER(FsCamera)), ("n_views", _I32), ("masks", _P),
                ("n_classes", _I32), ("A_hi", _P), ("A_lo", _P), ("S", _P), ("margin", _P), ("gamma", _F)]


class FsBatchOpts(ctypes.Structure):
    _fields_ = [("pair_budget", _I64), ("elem_budget", _I64), ("zero_accumulators", _I32), ("use_graph", _I32),
                ("reduction", _I32), ("depth_slabs", _I32), ("lanes", _I32)]


class FsBatchInfo(ctypes.Structure):
    _fields_ = [("n_chunks", _I32), ("n_views", _I32), ("pairs", _I64), ("pair_capacity", _I64),
                ("elements", _I64), ("tiles", _I64), ("workspace_bytes", _I64)]

    def as_dict(self):
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


class FsChunkInfo(ctypes.Structure):
    _fields_ = [("n_views", _I32), ("packed", _I32), ("n_tiles", _I64), ("n_pairs", _I64)]

    def as_dict(self):
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


# every symbol the header declares (checked by the CPU test)
EXPORTS = ["fs_version", "fs_error_string", "fs_params_default", "fs_params_exact", "fs_ctx_create",
           "fs_ctx_set_stream", "fs_ctx_destroy", "fs_ctx_last_error", "fs_status_get", "fs_project",
           "fs_bin_sort", "fs_accumulate", "fs_accumulate_noalloc", "fs_assign", "fs_assign_sweep", "fs_compact", "fs_render_masks",
           "fs_prompt_propagate", "fs_diagnose", "fs_last_accumulate_ms",
           "fs_batch_opts_default", "fs_batch_create",
           "fs_batch_run", "fs_batch_get_info", "fs_batch_destroy", "fs_batch_accumulate_ms",
           "fs_batch_chunk_lists"]

_lib = None


def load(path: str = LIB_PATH):
    """Load the library (after torch, so it binds to torch's HIP runtime)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"libflashsplat.so not found at {path}: run paper_2409_08270_amd/build.py "
                           "(or __graft_entry__.build()) first; there is no fallback")
    L = ctypes.CDLL(path)
    sig = {
        "fs_version": ([], ctypes.c_char_p),
        "fs_error_string": ([_I32], ctypes.c_char_p),
        "fs_params_default": ([ctypes.POINTER(FsParams)], None),
        "fs_params_exact": ([ctypes.POINTER(FsParams)], None),
        "fs_ctx_create": ([ctypes.POINTER(_P), _P], _I32),
        "fs_ctx_set_stream": ([_P, _P], _I32),
        "fs_ctx_destroy": ([_P], _I32),
        "fs_ctx_last_error": ([_P], ctypes.c_char_p),
        "fs_status_get": ([_P, ctypes.POINTER(FsStatus), _I32], _I32),
        "fs_project": ([_P, ctypes.POINTER(FsGaussians), ctypes.POINTER(FsCamera), _I32,
                        ctypes.POINTER(FsParams), ctypes.POINTER(FsProj)], _I32),
        "fs_bin_sort": ([_P, ctypes.POINTER(FsProj), ctypes.POINTER(FsCamera), ctypes.POINTER(FsParams),
                         ctypes.POINTER(FsBins), ctypes.POINTER(_I64)], _I32),
        "fs_accumulate": ([_P, ctypes.POINTER(FsProj), ctypes.POINTER(FsBins), ctypes.POINTER(FsCamera), _P, _I32,
                           ctypes.POINTER(FsParams), _P, _P, _I32, ctypes.POINTER(FsPixelOut)], _I32),
        "fs_accumulate_noalloc": ([_P, ctypes.POINTER(FsProj), ctypes.POINTER(FsBins), ctypes.POINTER(FsCamera), _P,
                                   _I32, ctypes.POINTER(FsParams), _P, _P, _I32, ctypes.POINTER(FsPixelOut)], _I32),
        "fs_assign": ([_P, _P, _P, _I64, _I32, _F, _P, _P], _I32),
        "fs_assign_sweep": ([_P, _P, _P, _I64, _I32, ctypes.POINTER(_F), _I32, _P, ctypes.POINTER(_I64)], _I32),
        "fs_compact": ([_P, ctypes.POINTER(FsGaussians), _P, _I32, ctypes.POINTER(FsGaussians), _P,
                        ctypes.POINTER(_I64)], _I32),
        "fs_render_masks": ([_P, ctypes.POINTER(FsProj), ctypes.POINTER(FsBins), ctypes.POINTER(FsCamera), _P, _I32,
                             ctypes.POINTER(FsParams), _F, _I32, _P, _P, _P], _I32),
        "fs_diagnose": ([_P, _P, _P, _P, _P, _I64, _I32, _F, _P, _P, _P], _I32),
        "fs_last_accumulate_ms": ([_P, ctypes.POINTER(_F)], _I32),
        "fs_prompt_propagate": ([_P, ctypes.POINTER(FsGaussians), ctypes.POINTER(FsCamera), _I32, _I32, _P, _I32,
                                 _I32, ctypes.POINTER(FsParams), _P, _P, _P, _P], _I32),
        "fs_batch_opts_default": ([ctypes.POINTER(FsBatchOpts)], None),
        "fs_batch_create": ([_P, ctypes.POINTER(FsScene), _I32, ctypes.POINTER(FsParams),
                             ctypes.POINTER(FsBatchOpts), ctypes.POINTER(_P)], _I32),
        "fs_batch_run": ([_P], _I32),
        "fs_batch_get_info": ([_P, ctypes.POINTER(FsBatchInfo)], _I32),
        "fs_batch_destroy": ([_P], _I32),
        "fs_batch_accumulate_ms": ([_P, ctypes.POINTER(_F), ctypes.POINTER(_I32)], _I32),
        "fs_batch_chunk_lists": ([_P, _I32, _P, _I64, _P, _I64, ctypes.POINTER(_I32), _I32,
                                  ctypes.POINTER(FsChunkInfo)], _I32),
    }
    for name, (args, res) in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    _lib = L
    return L


class FlashSplatError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{msg} (code {code})")
        self.code = code


def params(**over) -> FsParams:
    p = FsParams()
    load().fs_params_default(ctypes.byref(p))
    for k, v in over.items():
        setattr(p, k, v)
    return p


def params_exact(**over) -> FsParams:
    p = FsParams()
    load().fs_params_exact(ctypes.byref(p))
    for k, v in over.items():
        setattr(p, k, v)
    return p


def cameras(rows: np.ndarray):
    """FsCamera array from float32 [V, 18] rows (R9, t3, fx, fy, cx, cy, W, H)."""
    rows = np.asarray(rows, np.float32).reshape(-1, 18)
    arr = (FsCamera * rows.shape[0])()
    for i, r in enumerate(rows):
        arr[i].R[:] = [float(x) for x in r[0:9]]
        arr[i].t[:] = [float(x) for x in r[9:12]]
        arr[i].fx, arr[i].fy, arr[i].cx, arr[i].cy = [float(x) for x in r[12:16]]
        arr[i].width = int(r[16])
        arr[i].height = int(r[17])
    return arr


def _ptr(t: Optional[torch.Tensor]):
    if t is None:
        return None
    assert t.is_cuda and t.is_contiguous(), "device tensors must be contiguous and on the GPU"
    return ctypes.c_void_p(t.data_ptr())


class Context:
    """An fs_ctx bound to a torch stream (default: the current stream)."""

    def __init__(self, stream: Optional[torch.cuda.Stream] = None):
        self.L = load()
        self.stream = stream or torch.cuda.current_stream()
        h = _P()
        self._check(self.L.fs_ctx_create(ctypes.byref(h), _P(self.stream.cuda_stream)), ctx=None)
        self.h = h

    def _check(self, rc, ctx="self"):
        if rc != FS_OK:
            msg = self.L.fs_error_string(rc).decode()
            if ctx is not None and getattr(self, "h", None) is not None:
                last = self.L.fs_ctx_last_error(self.h).decode()
                if last:
                    msg = f"{msg}: {last}"
            raise FlashSplatError(rc, msg)
        return rc

    def close(self):
        if getattr(self, "h", None) is not None:
            self.L.fs_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def status(self, clear: bool = True, raise_on_error: bool = False) -> dict:
        st = FsStatus()
        rc = self.L.fs_status_get(self.h, ctypes.byref(st), 1 if clear else 0)
        if rc != FS_OK and (rc != FS_ERR_DEVICE or raise_on_error):
            self._check(rc)
        return st.as_dict()

    # -- the four calls ----------------------------------------------------
    def fs_project(self, gauss: "DeviceScene", cams, n_views: int, prm: FsParams, proj: "Proj"):
        return self._check(self.L.fs_project(self.h, ctypes.byref(gauss.struct()), cams, n_views,
                                             ctypes.byref(prm), ctypes.byref(proj.struct())))

    def fs_bin_sort(self, proj: "Proj", cams, prm: FsParams, bins: "Bins", sync_count: bool = True):
        n = _I64(0)
        rc = self.L.fs_bin_sort(self.h, ctypes.byref(proj.struct()), cams, ctypes.byref(prm),
                                ctypes.byref(bins.struct()), ctypes.byref(n) if sync_count else None)
        if rc == FS_ERR_CAPACITY:
            return -int(n.value)
        self._check(rc)
        return int(n.value) if sync_count else None

    def fs_accumulate(self, proj: "Proj", bins: "Bins", cams, masks: torch.Tensor, n_classes: int,
                      prm: FsParams, A_hi: torch.Tensor, A_lo: Optional[torch.Tensor],
                      reduction: int = FS_RED_AUTO, t_final: Optional[torch.Tensor] = None,
                      n_blend: Optional[torch.Tensor] = None):
        pix = None
        if t_final is not None or n_blend is not None:
            pix = FsPixelOut(_ptr(t_final), _ptr(n_blend))
        return self._check(self.L.fs_accumulate(self.h, ctypes.byref(proj.struct()), ctypes.byref(bins.struct()),
                                                cams, _ptr(masks), n_classes, ctypes.byref(prm), _ptr(A_hi),
                                                _ptr(A_lo), reduction, ctypes.byref(pix) if pix else None))

    def fs_accumulate_noalloc(self, proj: "Proj", bins: "Bins", cams, masks: torch.Tensor, n_classes: int,
                              prm: FsParams, A_hi: torch.Tensor, A_lo: Optional[torch.Tensor],
                              reduction: int = FS_RED_AUTO, t_final: Optional[torch.Tensor] = None,
                              n_blend: Optional[torch.Tensor] = None):
        """fs_accumulate with its workspace in the library's static scratch (allocates nothing)."""
        pix = None
        if t_final is not None or n_blend is not None:
            pix = FsPixelOut(_ptr(t_final), _ptr(n_blend))
        return self._check(self.L.fs_accumulate_noalloc(self.h, ctypes.byref(proj.struct()),
                                                        ctypes.byref(bins.struct()), cams, _ptr(masks), n_classes,
                                                        ctypes.byref(prm), _ptr(A_hi), _ptr(A_lo), reduction,
                                                        ctypes.byref(pix) if pix else None))

    def fs_assign(self, A_hi: torch.Tensor, A_lo: Optional[torch.Tensor], n: int, n_classes: int, gamma: float,
                  S: torch.Tensor, margin: Optional[torch.Tensor] = None):
        return self._check(self.L.fs_assign(self.h, _ptr(A_hi), _ptr(A_lo), n, n_classes, float(gamma), _ptr(S),
                                            _ptr(margin)))


    def fs_assign_sweep(self, A_hi: torch.Tensor, A_lo: Optional[torch.Tensor], n: int, n_classes: int, gammas,
                        S: Optional[torch.Tensor] = None, want_counts: bool = True):
        g = (_F * len(gammas))(*[float(x) for x in gammas])
        cnt = (_I64 * (len(gammas) * n_classes))() if want_counts else None
        self._check(self.L.fs_assign_sweep(self.h, _ptr(A_hi), _ptr(A_lo), n, n_classes, g, len(gammas), _ptr(S),
                                           cnt))
        return np.frombuffer(cnt, dtype=np.int64).reshape(len(gammas), n_classes).copy() if want_counts else None

    def fs_render_masks(self, proj: "Proj", bins: "Bins", cams, S: torch.Tensor, n_classes: int, prm: FsParams,
                        tau: float, mode: int, labels: torch.Tensor, rho: Optional[torch.Tensor] = None,
                        depth: Optional[torch.Tensor] = None):
        return self._check(self.L.fs_render_masks(self.h, ctypes.byref(proj.struct()), ctypes.byref(bins.struct()),
                                                  cams, _ptr(S), n_classes, ctypes.byref(prm), float(tau), int(mode),
                                                  _ptr(labels), _ptr(rho), _ptr(depth)))

    def fs_last_accumulate_ms(self) -> float:
        """Duration of the last fs_accumulate's compositing kernel (HIP events on the stream)."""
        ms = _F(0.0)
        self._check(self.L.fs_last_accumulate_ms(self.h, ctypes.byref(ms)))
        return float(ms.value)

    def fs_diagnose(self, A_hi, A_lo, S, gt, n: int, E: int, rel_eps: float = 0.0):
        """Returns (contrib_hist [E+1], member_hist [E+1], overlap [E, 3]) as uint64
        arrays; an entry whose inputs are None comes back as None."""
        c = np.zeros(E + 1, np.uint64) if A_hi is not None else None
        m = np.zeros(E + 1, np.uint64) if S is not None else None
        o = np.zeros((E, 3), np.uint64) if (S is not None and gt is not None) else None
        self._check(self.L.fs_diagnose(self.h, _ptr(A_hi), _ptr(A_lo), _ptr(S), _ptr(gt), n, E, float(rel_eps),
                                       None if c is None else c.ctypes.data, None if m is None else m.ctypes.data,
                                       None if o is None else o.ctypes.data))
        return c, m, o

    def fs_prompt_propagate(self, scene: "DeviceScene", ref_view: int, prompts, k: int = 10,
                            prm: Optional[FsParams] = None):
        """prompts: [P][3] (px, py, depth) on view ref_view. Returns (chosen int64 [P],
        nearest int64 [P, k], uv float32 [P, V, 2], visible uint8 [P, V])."""
        cams, nv = scene.cams()
        prm = prm or params()
        pr = np.ascontiguousarray(np.asarray(prompts, dtype=np.float32).reshape(-1, 3))
        P = pr.shape[0]
        chosen = np.zeros(P, np.int64)
        nearest = np.zeros((P, k), np.int64)
        uv = np.zeros((P, nv, 2), np.float32)
        vis = np.zeros((P, nv), np.uint8)
        self._check(self.L.fs_prompt_propagate(self.h, ctypes.byref(scene.struct()), cams, nv, ref_view,
                                               pr.ctypes.data, P, k, ctypes.byref(prm), chosen.ctypes.data,
                                               nearest.ctypes.data, uv.ctypes.data, vis.ctypes.data))
        return chosen, nearest, uv, vis

    def fs_compact(self, scene: "DeviceScene", select: torch.Tensor, keep_selected: bool,
                   capacity: Optional[int] = None, want_index: bool = True):
        """Returns (arrays: list of 11 device tensors, index_map or None)."""
        cap = scene.n if capacity is None else int(capacity)
        out = [torch.empty(max(1, cap), dtype=torch.float32, device=select.device) for _ in range(11)]
        idx = torch.empty(max(1, cap), dtype=torch.int64, device=select.device) if want_index else None
        o = FsGaussians(*[_ptr(a) for a in out], cap)
        n_out = _I64(0)
        self._check(self.L.fs_compact(self.h, ctypes.byref(scene.struct()), _ptr(select), 1 if keep_selected else 0,
                                      ctypes.byref(o), _ptr(idx), ctypes.byref(n_out)))
        k = int(n_out.value)
        return [a[:k] for a in out], (idx[:k] if idx is not None else None)


class DeviceScene:
    """A scene's Gaussians, cameras and masks resident on the GPU."""

    def __init__(self, scene, device="cuda"):
        self.n = scene.n
        self.E = scene.E
        self.arrays = [torch.from_numpy(np.ascontiguousarray(a)).to(device) for a in scene.gaussian_arrays()]
        self.cam_rows = scene.camera_rows()
        self.n_views = scene.n_views
        self.W = scene.W.copy()
        self.H = scene.H.copy()
        self.mask_off = np.concatenate([[0], np.cumsum(scene.W.astype(np.int64) * scene.H.astype(np.int64))])
        self.masks = torch.from_numpy(np.concatenate([m.reshape(-1) for m in scene.masks])).to(device)

    def struct(self) -> FsGaussians:
        g = FsGaussians(*[_ptr(a) for a in self.arrays], self.n)
        return g

    def cams(self, views: Optional[Sequence[int]] = None):
        rows = self.cam_rows if views is None else self.cam_rows[list(views)]
        return cameras(rows), rows.shape[0]

    def masks_of(self, v0: int, v1: int) -> torch.Tensor:
        return self.masks[int(self.mask_off[v0]):int(self.mask_off[v1])]

    def view_subset(self, views: Sequence[int]) -> "DeviceScene":
        """The same Gaussians (shared, not copied) seen from a subset of the
        views; the subset's masks are gathered into one buffer."""
        views = [int(v) for v in views]
        sub = DeviceScene.__new__(DeviceScene)
        sub.n, sub.E, sub.arrays = self.n, self.E, self.arrays
        sub.cam_rows = self.cam_rows[views]
        sub.n_views = len(views)
        sub.W, sub.H = self.W[views], self.H[views]
        sub.mask_off = np.concatenate([[0], np.cumsum(sub.W.astype(np.int64) * sub.H.astype(np.int64))])
        sub.masks = torch.cat([self.masks_of(v, v + 1) for v in views]) if views else self.masks[:0]
        return sub


class Proj:
    """Caller-owned fs_proj planes for n_views x n elements."""

    def __init__(self, n: int, n_views: int, device="cuda"):
        self.n, self.n_views = n, n_views
        self.rec = torch.empty((n_views, n, 8), dtype=torch.float32, device=device)
        self.rect = torch.empty((n_views, n, 4), dtype=torch.int16, device=device)
        self.ntiles = torch.empty((n_views, n), dtype=torch.int32, device=device)
        self.flags = torch.empty((n_views, n), dtype=torch.uint8, device=device)

    def struct(self) -> FsProj:
        return FsProj(_ptr(self.rec), _ptr(self.rect), _ptr(self.ntiles), _ptr(self.flags), self.n, self.n_views)


class Bins:
    def __init__(self, capacity: int, total_tiles: int, device="cuda"):
        self.capacity = int(capacity)
        self.vals = torch.empty(max(1, self.capacity), dtype=torch.int32, device=device)
        self.tiles = torch.empty(max(1, self.capacity), dtype=torch.int32, device=device)
        self.ranges = torch.empty((max(1, total_tiles), 2), dtype=torch.int32, device=device)

    def struct(self) -> FsBins:
        return FsBins(_ptr(self.vals), _ptr(self.tiles), _ptr(self.ranges), self.capacity)


def batch_opts(**over) -> FsBatchOpts:
    o = FsBatchOpts()
    load().fs_batch_opts_default(ctypes.byref(o))
    for k, v in over.items():
        setattr(o, k, v)
    return o


class Batch:
    """An fs_batch: many scenes solved by one graph launch.

    `scenes` are DeviceScene objects; the accumulators (A_hi, A_lo [n][E]),
    labels S [E][n] and optional margins are allocated here and borrowed by
    the library until close(). `gammas` gives one background bias per scene.
    """

    def __init__(self, ctx: Context, scenes: Sequence["DeviceScene"], prm: FsParams,
                 gammas: Optional[Sequence[float]] = None, compensated: bool = True, want_labels: bool = True,
                 want_margin: bool = False, **opts):
        self.ctx = ctx
        self.L = ctx.L
        self.scenes = list(scenes)
        dev = ctx.stream.device
        self.A_hi, self.A_lo, self.S, self.margin, self._cams = [], [], [], [], []
        arr = (FsScene * len(self.scenes))()
        for i, ds in enumerate(self.scenes):
            n, E = ds.n, ds.E
            self.A_hi.append(torch.zeros((n, E), dtype=torch.float32, device=dev))
            self.A_lo.append(torch.zeros((n, E), dtype=torch.float32, device=dev) if compensated else None)
            self.S.append(torch.zeros((E, n), dtype=torch.uint8, device=dev) if want_labels else None)
            self.margin.append(torch.zeros((E, n), dtype=torch.float32, device=dev) if want_margin else None)
            cams, nv = ds.cams()
            self._cams.append(cams)
            g = 0.0 if gammas is None else float(gammas[i])
            arr[i] = FsScene(ds.struct(), ctypes.cast(cams, ctypes.POINTER(FsCamera)), nv, _ptr(ds.masks), E,
                             _ptr(self.A_hi[i]), _ptr(self.A_lo[i]), _ptr(self.S[i]), _ptr(self.margin[i]), g)
        o = batch_opts(**opts)
        h = _P()
        ctx._check(self.L.fs_batch_create(ctx.h, arr, len(self.scenes), ctypes.byref(prm), ctypes.byref(o),
                                          ctypes.byref(h)))
        self.h = h

    def run(self):
        self.ctx._check(self.L.fs_batch_run(self.h))

    def info(self) -> dict:
        inf = FsBatchInfo()
        self.ctx._check(self.L.fs_batch_get_info(self.h, ctypes.byref(inf)))
        return inf.as_dict()

    def accumulate_ms(self):
        """(total ms, launches) of the compositing launches of the last run (batches without a graph)."""
        ms, cnt = _F(0.0), _I32(0)
        self.ctx._check(self.L.fs_batch_accumulate_ms(self.h, ctypes.byref(ms), ctypes.byref(cnt)))
        return float(ms.value), int(cnt.value)

    def chunk_lists(self, chunk: int):
        """The tile lists the solve builds for one chunk: (info, vals [n_pairs] u32 numpy,
        ranges [n_tiles, 2] u32 numpy, view refs [(scene, view)])."""
        inf = FsChunkInfo()
        self.ctx._check(self.L.fs_batch_chunk_lists(self.h, chunk, None, 0, None, 0, None, 0, ctypes.byref(inf)))
        dev = self.ctx.stream.device
        vals = torch.empty(max(1, inf.n_pairs), dtype=torch.int32, device=dev)
        ranges = torch.empty((max(1, inf.n_tiles), 2), dtype=torch.int32, device=dev)
        refs = (_I32 * (2 * max(1, inf.n_views)))()
        self.ctx._check(self.L.fs_batch_chunk_lists(self.h, chunk, _ptr(vals), vals.numel(), _ptr(ranges),
                                                    ranges.shape[0], refs, inf.n_views, ctypes.byref(inf)))
        v = vals[:inf.n_pairs].cpu().numpy().view(np.uint32)
        r = ranges[:inf.n_tiles].cpu().numpy().view(np.uint32)
        rr = [(refs[2 * j], refs[2 * j + 1]) for j in range(inf.n_views)]
        return inf.as_dict(), v, r, rr

    def close(self):
        if getattr(self, "h", None) is not None:
            self.L.fs_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
