"""Tuner for the batched solve (fs_batch): picks, per workload, the tile
shape, compositing work order, compositing launch (one workgroup per tile or
resident workgroups pulling tiles from a counter), LDS batch depth, depth
slabs, reduction strategy and number of lanes that give the shortest graph
replay, among
settings whose result agrees with the library's defaults. The defaults are
kept unless a setting is at least `min_gain` faster, so that timing noise does
not decide. By default the compensated reductions (LDS pre-reduction +
two-sum into A_lo, and the bit-reproducible fixed-point sums) are candidates;
`compensated=False` also tries the LDS pre-reduction without A_lo.

The support of a splat is an ellipse, so A does not depend on the tile shape,
the work order, the launch shape or the batch depth beyond floating-point
summation order (Eq. (7) sums the same weights); a candidate is kept only if
its A agrees with the reference run's within `rel` (aggregate L1) and its
labels are identical wherever the reference's margin is at least `margin`.

Search: `search="staged"` (default) tunes one setting at a time in the order
of KNOBS, starting from the defaults and keeping the best value of each
before moving to the next; `search="all"` times every combination.

The table is JSON: {"version": 1, "entries": {key: {"params": {...},
"opts": {...}, "ms": t, "reference_ms": t0, "candidates": [...]}}}, keyed by
`batch_key` (one scene: classes, image size, Gaussian-count bucket, views;
several: scene count, Gaussian and pixel buckets, views, classes).
Timing runs on the GPU; the keys, the candidate lists and the table I/O are
plain Python.
"""
import itertools
import json
import os
import time
from typing import Iterable, List, Optional, Sequence

TABLE_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuned.json")


def _bucket(n: int) -> int:
    b = 1
    while b < n:
        b <<= 1
    return b


def workload_key(n_gaussians: int, width: int, height: int, n_classes: int, n_views: int) -> str:
    """Table key: classes, image size, Gaussian count rounded up to a power of two, views."""
    return f"E{int(n_classes)}-{int(width)}x{int(height)}-N{_bucket(int(n_gaussians))}-V{int(n_views)}"


def scene_key(scene) -> str:
    return workload_key(scene.n, int(scene.W[0]), int(scene.H[0]), scene.E, scene.n_views)


def batch_key(scenes) -> str:
    """Table key of a batch: one scene's key, or for several scenes their count, total
    Gaussians and pixels (rounded up to powers of two), total views and largest class count."""
    scenes = list(scenes)
    if len(scenes) == 1:
        return scene_key(scenes[0])
    n = sum(int(s.n) for s in scenes)
    px = sum(int(s.pixels()) for s in scenes)
    return (f"B{len(scenes)}-N{_bucket(n)}-P{_bucket(px)}-V{sum(int(s.n_views) for s in scenes)}"
            f"-E{max(int(s.E) for s in scenes)}")


# tunable settings in search order: (table section, name, values); "tile" sets tile_w x tile_h
KNOBS = [("opts", "lanes", [1, 2, 3, 4]),
         ("params", "tile", [(16, 16), (32, 8), (8, 32)]),
         ("params", "tile_order", [0, 1]),
         ("params", "persistent", [0, 1]),
         ("params", "lds_batch", [256, 128, 64]),
         ("opts", "depth_slabs", [1, 2, 3]),
         ("opts", "reduction", None)]  # None: the reductions allowed by `compensated`


def _reductions(compensated: bool):
    from . import _lib as L
    # FS_RED_DET (fixed-point sums, bit-reproducible) keeps A_lo compensated too
    return [L.FS_RED_LDS2SUM, L.FS_RED_DET] if compensated else [L.FS_RED_LDS2SUM, L.FS_RED_LDS, L.FS_RED_DET]


def reference() -> dict:
    """The library's defaults (16x16 tiles, longest list first, one workgroup per tile,
    256-entry LDS batches, one depth slab, LDS + two-sum, 2 lanes)."""
    from . import _lib as L
    return {"params": {"tile_w": 16, "tile_h": 16, "tile_order": 0, "persistent": 0, "lds_batch": 256},
            "opts": {"reduction": L.FS_RED_LDS2SUM, "lanes": 2, "depth_slabs": 1}}


def _with(c: dict, sec: str, name: str, value) -> dict:
    out = {"params": dict(c["params"]), "opts": dict(c["opts"])}
    if name == "tile":
        out["params"]["tile_w"], out["params"]["tile_h"] = value
    else:
        out[sec][name] = value
    return out


def candidates(width: int = 0, height: int = 0, compensated: bool = True) -> List[dict]:
    """Every combination of the tunable settings (256-pixel tiles)."""
    ref = reference()
    lists = [(sec, name, vals if vals is not None else _reductions(compensated)) for sec, name, vals in KNOBS]
    out = []
    for combo in itertools.product(*[v for _, _, v in lists]):
        c = ref
        for (sec, name, _), val in zip(lists, combo):
            c = _with(c, sec, name, val)
        out.append(c)
    return out


def _same(a: dict, b: dict) -> bool:
    return a["params"] == b["params"] and a["opts"] == b["opts"]


def tune(scenes, cands: Optional[Sequence[dict]] = None, steps: int = 4, warmup: int = 1, rel: float = 2e-5,
         margin: float = 1e-4, min_gain: float = 0.01, compensated: bool = True, search: str = "staged",
         log=None) -> dict:
    """Times settings on `scenes` (one scenegen Scene or a list, solved as one batch) and
    returns the table entry. With `cands` given, exactly those are timed (the first
    is the reference); otherwise `search` decides."""
    import numpy as np
    import torch
    from . import _lib as L

    scenes = list(scenes) if isinstance(scenes, (list, tuple)) else [scenes]
    ctx = L.Context()
    dss = [L.DeviceScene(s) for s in scenes]
    gam = [0.0] * len(scenes)

    def run(c, want_margin):
        prm = L.params(count_ops=0, **c["params"])
        b = L.Batch(ctx, dss, prm, gammas=gam, want_margin=want_margin, **c["opts"])
        for _ in range(warmup):
            b.run()
        torch.cuda.synchronize()
        best = float("inf")
        for _ in range(2):
            t = time.perf_counter()
            for _ in range(steps):
                b.run()
            torch.cuda.synchronize()
            best = min(best, (time.perf_counter() - t) / steps)
        A, S, M = [], [], []
        for i in range(len(scenes)):
            a = b.A_hi[i].double()
            if b.A_lo[i] is not None:
                a = a + b.A_lo[i].double()
            A.append(a.cpu().numpy())
            S.append(b.S[i].cpu().numpy())
            M.append(b.margin[i].cpu().numpy() if want_margin else None)
        b.close()
        ctx.status()
        return {"A": A, "S": S, "margin": M, "ms": best * 1e3}

    base = None
    rows = []

    def measure(c):
        nonlocal base
        for r in rows:
            if _same(r, c):
                return r
        try:
            r = run(c, base is None)
        except L.FlashSplatError as err:  # a setting the library rejects for this workload
            row = {**c, "ms": None, "a_rel": None, "label_flips": None, "valid": False, "error": str(err)}
            rows.append(row)
            if log:
                log(f"[tune] {c['params']} {c['opts']}: rejected by the library ({err})")
            return row
        if base is None:
            base = r
        s_ref = sum(np.abs(a).sum() for a in base["A"])
        d = float(sum(np.abs(a - a0).sum() for a, a0 in zip(r["A"], base["A"])) / max(s_ref, 1e-300))
        flips = int(sum(((x != x0) & ~(m0 < margin)).sum() for x, x0, m0 in zip(r["S"], base["S"], base["margin"])))
        ok = d <= rel and flips == 0
        row = {**c, "ms": r["ms"], "a_rel": d, "label_flips": flips, "valid": ok}
        rows.append(row)
        if log:
            log(f"[tune] {c['params']} {c['opts']}: {r['ms']:.3f} ms, A rel {d:.2e}, flips {flips}"
                f"{'' if ok else ' (rejected)'}")
        return row

    if cands is not None:
        for c in list(cands):
            measure(c)
        best = min((r for r in rows if r["valid"]), key=lambda r: r["ms"])
    else:
        best = measure(reference())
        if search == "all":
            for c in candidates(compensated=compensated):
                measure(c)
            best = min((r for r in rows if r["valid"]), key=lambda r: r["ms"])
        else:
            cur = reference()
            for sec, name, vals in KNOBS:
                for v in (vals if vals is not None else _reductions(compensated)):
                    r = measure(_with(cur, sec, name, v))
                    if r["valid"] and r["ms"] < best["ms"] * (1.0 - min_gain):
                        best = r
                cur = {"params": dict(best["params"]), "opts": dict(best["opts"])}
    if best["ms"] > rows[0]["ms"] * (1.0 - min_gain):
        best = rows[0]  # not clearly faster than the reference
    ctx.close()
    return {"params": best["params"], "opts": best["opts"], "ms": best["ms"], "reference_ms": rows[0]["ms"],
            "candidates": rows}


def load(path: str = TABLE_PATH) -> dict:
    if not os.path.exists(path):
        return {"version": 1, "entries": {}}
    with open(path) as f:
        t = json.load(f)
    if t.get("version") != 1 or not isinstance(t.get("entries"), dict):
        raise ValueError(f"{path}: not a tuning table")
    return t


def save(table: dict, path: str = TABLE_PATH) -> None:
    with open(path, "w") as f:
        json.dump(table, f, indent=1, sort_keys=True)
        f.write("\n")


def lookup(table: dict, key: str) -> Optional[dict]:
    """The tuned {"params", "opts"} for a workload key, or None."""
    e = table.get("entries", {}).get(key)
    if e is None:
        return None
    return {"params": dict(e["params"]), "opts": dict(e["opts"])}


def main(argv: Optional[Iterable[str]] = None) -> int:
    import argparse
    import sys
    ap = argparse.ArgumentParser(description="tune the batched solve for synthetic workloads")
    ap.add_argument("--config", action="append", default=None,
                    help="scenegen config, C1-C4 or C5 (the 32-scene batch); repeatable; default C2")
    ap.add_argument("--out", default=TABLE_PATH, help="table to update")
    ap.add_argument("--steps", type=int, default=4)
    ap.add_argument("--search", default="staged", choices=["staged", "all"])
    ap.add_argument("--uncompensated", action="store_true", help="also try the reduction without two-sum")
    args = ap.parse_args(list(argv) if argv is not None else None)
    import scenegen as sg
    table = load(args.out) if os.path.exists(args.out) else {"version": 1, "entries": {}}
    for name in args.config or ["C2"]:
        scenes = sg.make_batch(32) if name == "C5" else [sg.make_config(name)]
        key = batch_key(scenes)
        e = tune(scenes, steps=args.steps, compensated=not args.uncompensated, search=args.search,
                 log=lambda m: print(m, file=sys.stderr, flush=True))
        e["workload"] = name
        table["entries"][key] = e
        save(table, args.out)
        print(f"[tune] {name} -> {key}: {e['params']} {e['opts']} {e['ms']:.3f} ms "
              f"(defaults {e['reference_ms']:.3f} ms)", flush=True)
    return 0


if __name__ == "__main__":
    raise SystemExit(main())
