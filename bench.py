#!/usr/bin/env python3
"""Throughput of the splat-and-accumulate path on one MI355X.

Workload: the 200k-Gaussian plain configuration (4 clustered objects plus a
background shell, 50 orbit views at 640x480, binary masks with boundary
erosion, background bias 0), synthetic and seeded. One step = one full solve:
project, bin/sort, composite + accumulate over all 50 views, then assign.

Prints one JSON line: views/s of the batched path (value), blends/s, the
plain per-view path for comparison, the roofline of the compositing kernel,
and the CPU oracle timed on a bounded sample of views.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_ALU_OPS = 256 * 64 * 2.4e9   # fp32 lane-ops/s: 256 CUs x 64 lanes/clk x 2.4 GHz (no packed, no FMA credit)
PEAK_HBM = 8.0e12


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", default="C2")
    ap.add_argument("--cpu-views", type=int, default=24, help="views of the CPU oracle sample (0: skip)")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--lanes", type=int, default=0, help="batch lanes (0: the tuned or the library's default)")
    ap.add_argument("--tuned", default=None, help="tuning table (default: the package's tuned.json)")
    ap.add_argument("--no-tuned", action="store_true", help="run the library's default settings")
    ap.add_argument("--no-strategies", action="store_true",
                    help="skip the per-strategy compositing comparison (keeps one launch shape per kernel)")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run a device-to-device copy of this many MiB (HBM counter calibration)")
    return ap.parse_args()


def recorded_traffic():
    """HBM bytes per compositing launch from the committed rocprofv3 FETCH_SIZE / WRITE_SIZE
    summary (scaled by the copy-probe calibration), or None when the kernel source has changed
    since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "k_accum_c2_traffic.json")
    try:
        rec = json.load(open(path))
    except (OSError, ValueError):
        return None
    csrc = os.path.join(ROOT, "paper_2409_08270_amd", "csrc")
    src = open(os.path.join(csrc, "fs_accum.hip"), "rb").read() + open(os.path.join(csrc, "fs_internal.h"), "rb").read()
    if hashlib.sha256(src).hexdigest() != rec.get("kernel_source_sha256"):
        return None
    return float(rec["hbm_bytes_per_launch"])


def copy_probe(mib: int):
    """A plain copy of known size: its FETCH_SIZE / WRITE_SIZE readings give the
    factor between those counters and real HBM bytes."""
    import torch
    torch.cuda.set_device(0)
    n = mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes_each_way": n * 4, "launches": 3}))


def main():
    args = parse()
    if args.copy_probe:
        copy_probe(args.copy_probe)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print(json.dumps({"error": "this program runs on exactly one GPU; multi-GPU runs are not supported "
                                   "(views would shard across GPUs with one reduce-scatter of A)"}))
        sys.exit(2)
    import numpy as np
    import torch

    import scenegen as sg
    from paper_2409_08270_amd import _lib as L
    from paper_2409_08270_amd.solve import Solver

    torch.cuda.set_device(0)
    t0 = time.time()
    sc = sg.make_config(args.config)
    print(f"[bench] scene {args.config}: N={sc.n} views={sc.n_views} {int(sc.W[0])}x{int(sc.H[0])} E={sc.E} "
          f"(generated in {time.time() - t0:.1f}s)", file=sys.stderr, flush=True)
    ds = L.DeviceScene(sc)
    ctx = L.Context()
    V = sc.n_views

    # settings of the batched solve: the tuner's entry for this workload shape, if any
    from paper_2409_08270_amd import tune as T
    tuned = None if args.no_tuned else T.lookup(T.load(args.tuned or T.TABLE_PATH), T.scene_key(sc))
    prm_kw = dict(tuned["params"]) if tuned else {}
    opt_kw = dict(tuned["opts"]) if tuned else {}
    if args.lanes:
        opt_kw["lanes"] = args.lanes
    print(f"[bench] settings: {'tuned ' + str(tuned) if tuned else 'library defaults'}; overrides {opt_kw}",
          file=sys.stderr, flush=True)

    # ---- batched: the whole solve (all views, assignment included) as one graph launch ----
    # The timed graph runs without the per-step evaluation/blend counters (count_ops = 0:
    # same A and S, two fewer instructions per pixel step); the work it does is counted by
    # one replay of an instrumented graph of the same workload.
    prm = L.params(count_ops=0, **prm_kw)
    prm_count = L.params(count_ops=1, **prm_kw)
    counted = L.Batch(ctx, [ds], prm_count, gammas=[0.0], **opt_kw)
    ctx.status()
    counted.run()
    torch.cuda.synchronize()
    st = ctx.status()
    S_counted = counted.S[0].cpu().numpy()
    counted.close()
    del counted
    blends = float(st["blends"])
    evals = float(st["evaluated"])
    staged = float(st["entries_staged"])
    wsteps, wsteps_max = float(st["wave_steps"]), float(st["wave_steps_max"])
    batch = L.Batch(ctx, [ds], prm, gammas=[0.0], **opt_kw)
    binfo = batch.info()
    print(f"[bench] batch planned: {binfo}", file=sys.stderr, flush=True)
    for _ in range(args.warmup):
        batch.run()
    torch.cuda.synchronize()
    ctx.status()
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(args.steps):
        batch.run()
    torch.cuda.synchronize()
    dt_b = (time.perf_counter() - t) / args.steps
    st_t = ctx.status()
    assert st_t["blends"] == 0 and st_t["evaluated"] == 0, "the timed graph was not the uncounted one"
    labels_differ = int((batch.S[0].cpu().numpy() != S_counted).sum())
    pairs_emitted = st_t["pairs_emitted"] / args.steps
    pairs = binfo["pairs"]

    # ---- the compositing kernel alone, same launch as inside the graph, timed with HIP events
    # recorded on the stream it runs on
    solver = Solver(ctx, ds, prm)
    solver.solve(chunk=V, want_margin=False)
    cams, nv = ds.cams()
    n, E = sc.n, sc.E
    A_hi = torch.zeros((n, E), dtype=torch.float32, device="cuda")
    A_lo = torch.zeros((n, E), dtype=torch.float32, device="cuda")
    ctx.status()
    ctx.fs_accumulate(solver.proj, solver.bins, cams, ds.masks, E, prm_count, A_hi, A_lo, L.FS_RED_LDS2SUM)
    st_acc = ctx.status()
    assert abs(st_acc["blends"] - blends) <= 1e-6 * blends, "standalone compositing saw different work than the graph"
    acc_ms = []
    for _ in range(args.steps):
        # HIP events that the library records on its stream right around the compositing launch
        ctx.fs_accumulate(solver.proj, solver.bins, cams, ds.masks, E, prm, A_hi, A_lo, L.FS_RED_LDS2SUM)
        acc_ms.append(ctx.fs_last_accumulate_ms())
    print(f"[bench] batched graph: {dt_b * 1e3:.2f} ms/step, pairs planned {pairs} sorted {pairs_emitted:.0f}, "
          f"blends {blends:.3e}, "
          f"evaluated {evals:.3e}, accumulate kernel {np.mean(acc_ms):.3f} ms; wave steps {wsteps:.3e}, "
          f"4 x per-tile max {4 * wsteps_max:.3e}", file=sys.stderr, flush=True)

    # ---- compositing kernel alone, per reduction strategy (same bins) --------
    strat = {}
    prm_img = L.params(tile_order=1, count_ops=0)
    prm_xcd = L.params(tile_order=2, count_ops=0)
    for name, red, comp, prm_s in (() if args.no_strategies else (("plain_atomics", L.FS_RED_PLAIN, False, prm),
                                 ("lds", L.FS_RED_LDS, False, prm),
                                 ("lds_two_sum", L.FS_RED_LDS2SUM, True, prm),
                                 ("lds_two_sum_image_order", L.FS_RED_LDS2SUM, True, prm_img),
                                 ("lds_two_sum_xcd_runs", L.FS_RED_LDS2SUM, True, prm_xcd))):
        n, E = sc.n, sc.E
        A_hi = torch.zeros((n, E), dtype=torch.float32, device="cuda")
        A_lo = torch.zeros((n, E), dtype=torch.float32, device="cuda") if comp else None
        ts = []
        for _ in range(3):
            ctx.fs_accumulate(solver.proj, solver.bins, cams, ds.masks, E, prm_s, A_hi, A_lo, red)
            ts.append(ctx.fs_last_accumulate_ms())
        strat[name] = float(np.median(ts))
    ctx.status()
    print(f"[bench] compositing kernel per strategy (ms): {strat}", file=sys.stderr, flush=True)

    # ---- plain (per view) ---------------------------------------------------
    dt_p = None
    if not args.no_plain:
        for _ in range(max(1, args.warmup // 2)):
            solver.solve(chunk=1, want_margin=False)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(args.steps):
            solver.solve(chunk=1, want_margin=False)
        torch.cuda.synchronize()
        dt_p = (time.perf_counter() - t) / args.steps
        ctx.status()
        print(f"[bench] plain: {dt_p * 1e3:.2f} ms/step", file=sys.stderr, flush=True)

    # ---- follow-ups once A is known: bias sweep, object removal ----------------
    def timed(fn, reps=5):
        ts = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(ctx.stream)
            fn()
            e1.record(ctx.stream)
            e1.synchronize()
            ts.append(e0.elapsed_time(e1))
        return float(np.median(ts))

    S_one = torch.empty((sc.E, sc.n), dtype=torch.uint8, device="cuda")
    m_one = torch.empty((sc.E, sc.n), dtype=torch.float32, device="cuda")
    assign_ms = timed(lambda: ctx.fs_assign(batch.A_hi[0], batch.A_lo[0], sc.n, sc.E, 0.0, S_one, m_one))
    gam = [float(x) for x in np.linspace(-0.5, 0.5, 64)]
    S_sw = torch.empty((64, sc.E, sc.n), dtype=torch.uint8, device="cuda")
    sweep_ms = timed(lambda: ctx.fs_assign_sweep(batch.A_hi[0], batch.A_lo[0], sc.n, sc.E, gam, S_sw,
                                                 want_counts=False))
    sel = batch.S[0][1].contiguous()
    compact_ms = timed(lambda: ctx.fs_compact(ds, sel, False))
    labels = torch.empty(sc.pixels(), dtype=torch.uint8, device="cuda")
    render_ms = timed(lambda: ctx.fs_render_masks(solver.proj, solver.bins, cams, batch.S[0], sc.E, prm, 0.1,
                                                  L.FS_MASK_DEPTH, labels))
    agree = float((labels.cpu().numpy() == ds.masks.cpu().numpy()).mean())
    # point-prompt propagation (synchronous call: wall clock, host copies included)
    rng = np.random.default_rng(11)
    prompts = np.stack([rng.uniform(0, sc.W[0], 16), rng.uniform(0, sc.H[0], 16),
                        rng.uniform(2.0, 5.0, 16)], 1).astype(np.float32)
    ctx.fs_prompt_propagate(ds, 0, prompts, k=10)
    pts = []
    for _ in range(5):
        t = time.perf_counter()
        ctx.fs_prompt_propagate(ds, 0, prompts, k=10)
        pts.append((time.perf_counter() - t) * 1e3)
    followups = {"assign_ms": assign_ms, "prompt_propagation_16_prompts_ms": float(np.median(pts)), "bias_sweep_64_gammas_ms": sweep_ms, "object_removal_compaction_ms": compact_ms,
                 "mask_render_all_views_ms": render_ms, "mask_render_views_per_sec": V / (render_ms * 1e-3),
                 "rendered_masks_agree_with_inputs": agree, "gaussians": sc.n}
    print(f"[bench] follow-ups: {followups}", file=sys.stderr, flush=True)

    # ---- roofline of the compositing kernel (one launch over all views) -----
    # algorithmic fp32 ops: 15 per (pixel, Gaussian) pair inside the support (offset, quadratic form,
    # support test, exp, opacity, clamp, alpha test) + 5 per blend (1-alpha, T update, stop test, w, add)
    ops = 15.0 * evals + 5.0 * blends
    acc_s = float(np.mean(acc_ms)) * 1e-3
    achieved = ops / acc_s
    roof = {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_ALU_OPS / 1e12, "unit": "TFLOP/s",
            "frac": achieved / PEAK_ALU_OPS,
            # the counters were taken on 16x16 tiles in the longest-first order
            "traffic": recorded_traffic() if (prm.tile_w, prm.tile_h, prm.tile_order) == (16, 16, 0) else None,
            "traffic_unit": "bytes per launch (HBM)",
            "kernel": "k_accum",
            "ops_per_launch": ops, "launch_ms": acc_s * 1e3,
            "wave_steps": wsteps, "wave_balance": wsteps / max(1.0, 4 * wsteps_max)}

    # ---- the whole path against the HBM roof --------------------------------
    # algorithmic bytes of one step (what the method must move, from counted quantities):
    # Gaussians read once per chunk, 44 B per (Gaussian, view) for the projected record and its
    # count, 36 B per pair (emit + one sort read and write), 8 B per tile range, 28 B per staged
    # list entry (id + gathered record), the masks, and A written, read and S written once
    n_chunks = binfo["n_chunks"]
    terms = {"gaussians": 44.0 * sc.n * n_chunks, "projected": 44.0 * sc.n * V, "pairs": 36.0 * pairs,
             "ranges": 8.0 * binfo["tiles"], "staged": 28.0 * staged, "masks": float(sc.pixels()),
             "assign": 17.0 * sc.n * sc.E}
    path_bytes = sum(terms.values())
    hbm_frac = path_bytes / dt_b / PEAK_HBM
    path = {"hbm": {"algorithmic_bytes_per_step": path_bytes, "achieved": path_bytes / dt_b / 1e9,
                    "peak": PEAK_HBM / 1e9, "unit": "GB/s", "frac": hbm_frac, "terms": terms,
                    "entries_staged": staged},
            "alu_compositing_frac": roof["frac"],
            "binding": "alu (compositing)" if roof["frac"] >= hbm_frac else "hbm"}

    # ---- CPU oracle on a bounded sample of views -----------------------------
    cpu = None
    parity = None
    if args.cpu_views > 0:
        import oracle as O
        sample = [int(round(i * V / args.cpu_views)) for i in range(args.cpu_views)]
        cores = len(os.sched_getaffinity(0))
        os.environ.setdefault("OMP_NUM_THREADS", str(cores))
        t = time.perf_counter()
        ref = O.solve64(sc, O.params(), views=sample)
        dt_c = time.perf_counter() - t
        cpu = {"value": len(sample) / dt_c, "unit": "views/s", "cores": int(os.environ.get("OMP_NUM_THREADS", cores)),
               "kind": "oracle", "sample": f"views {sample} of {args.config} (binning in binary32 + compositing "
                                           f"and accumulation in binary64), {dt_c:.1f}s",
               "blends_per_sec": ref["blends"] / dt_c}
        # parity of the GPU path on the same views
        n, E = sc.n, sc.E
        A_hi = torch.zeros((n, E), dtype=torch.float32, device="cuda")
        A_lo = torch.zeros((n, E), dtype=torch.float32, device="cuda")
        s2 = Solver(ctx, ds)
        for v in sample:
            s2.accumulate_views([v], A_hi, A_lo)
        A = (A_hi.double() + A_lo.double()).cpu().numpy()
        d = np.abs(A - ref["A"]).sum(1)
        s = np.abs(ref["A"]).sum(1)
        bad = d > 1e-4 * s + ref["slack"] + 1e-9
        S64, m64 = O.assign64(ref["A"], 0.0)
        S_g = torch.empty((E, n), dtype=torch.uint8, device="cuda")
        ctx.fs_assign(A_hi, A_lo, n, E, 0.0, S_g, None)
        mism = int(((S_g.cpu().numpy() != S64) & (m64 >= 1e-4)).sum())
        parity = {"views": sample, "rows_off_tolerance": int(bad.sum()), "aggregate_rel": float(d.sum() / s.sum()),
                  "label_mismatches_margin_ge_1e-4": mism, "low_margin_entries": int((m64 < 1e-4).sum())}

    res = {
        "metric": "views/sec + Gaussian-pixel blends/sec; batched vs plain, labels matching oracle",
        "value": V / dt_b,
        "unit": "views/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt_b * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{args.config}: {sc.n} Gaussians (4 clusters + shell), {V} views "
                               f"{int(sc.W[0])}x{int(sc.H[0])}, E={sc.E}, gamma=0", "mode": "batched, one hipGraph",
                   "reduction": {L.FS_RED_LDS: "lds", L.FS_RED_LDS2SUM: "lds+two-sum"}.get(
                       opt_kw.get("reduction", L.FS_RED_LDS2SUM), "lds+two-sum"),
                   "chunks": binfo["n_chunks"], "lanes": opt_kw.get("lanes", 2),
                   "tile": f"{prm.tile_w}x{prm.tile_h}", "tile_order": int(prm.tile_order),
                   "settings": "tuned" if tuned else "library defaults"},
        "blends_per_sec": blends / dt_b,
        "op_counts": "timed graph and compositing launches run with count_ops=0; evaluations and blends "
                     "come from one instrumented replay of the same workload",
        "labels_differ_instrumented_vs_timed": labels_differ,
        "pairs_planned_per_step": pairs,
        "pairs_sorted_per_step": pairs_emitted,
        "depth_slabs": 1,
        "plain_views_per_sec": (V / dt_p) if dt_p else None,
        "batched_over_plain": (dt_p / dt_b) if dt_p else None,
        "accumulate_ms_by_strategy": strat,
        "followups": followups,
        "roofline": roof,
        "path_roofline": path,
        "cpu_baseline": cpu,
        "parity_sample": parity,
    }
    print(json.dumps(res))


if __name__ == "__main__":
    main()
