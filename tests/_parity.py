"""Comparison rules between the GPU library and the CPU oracle (tests only).

A (per-Gaussian, per-class contribution sums): for every row g,
    |A_gpu[g] - A64[g]|_1 <= REL * |A64[g]|_1 + slack[g] + ABS
where slack[g] is the oracle's budget for float32-vs-float64 threshold
decisions (alpha_min, t_min, support) that lie within its band; the
aggregate |dA|_1 / |A64|_1 must also stay within REL. REL = 1e-4 is the
acceptance tolerance for A.

Labels: S_gpu == S64 wherever the oracle's margin >= 1e-4, except where
the row's observed difference in A accounts for the flip (see
compare_labels); both kinds of excluded entries are counted and reported.
"""
import sys

import numpy as np

REL = 1e-4
ABS = 1e-9
MARGIN = 1e-4


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def compare_A(A_gpu: np.ndarray, A64: np.ndarray, slack: np.ndarray, rel: float = REL):
    A_gpu = np.asarray(A_gpu, np.float64)
    d = np.abs(A_gpu - A64).sum(axis=1)
    s = np.abs(A64).sum(axis=1)
    tol = rel * s + slack + ABS
    bad = d > tol
    seen = s > 0
    r = np.zeros_like(d)
    r[seen] = d[seen] / s[seen]
    clean = seen & (slack <= 1e-6 * s)
    stats = dict(rows=int(A64.shape[0]), seen=int(seen.sum()), rows_failing=int(bad.sum()),
                 rows_with_slack=int((slack > 0).sum()),
                 rows_over_rel_without_slack=int((d > rel * s + ABS).sum()),
                 max_rel=float(r.max()) if r.size else 0.0,
                 p99_rel=float(np.percentile(r[seen], 99)) if seen.any() else 0.0,
                 median_rel=float(np.median(r[seen])) if seen.any() else 0.0,
                 max_rel_clean=float(r[clean].max()) if clean.any() else 0.0,
                 aggregate_rel=float(d.sum() / max(s.sum(), 1e-300)))
    return stats, bad


def assert_A(A_gpu, A64, slack, rel=REL, what=""):
    st, bad = compare_A(A_gpu, A64, slack, rel)
    log(f"[A parity{(' ' + what) if what else ''}] {st}")
    if bad.any():
        idx = np.nonzero(bad)[0][:10]
        for g in idx:
            log(f"  row {g}: gpu {A_gpu[g]} oracle {A64[g]} slack {slack[g]}")
    assert st["rows_failing"] == 0, st
    assert st["aggregate_rel"] <= rel, st
    return st


def compare_labels(S_gpu, S64, margin64, A64=None, A_gpu=None):
    """Label parity. Entries whose oracle margin is below 1e-4 are excluded and
    counted. With the two A's given, a mismatch is also excused, and counted
    apart, where the row's observed difference alone moves the margin past
    zero: the margin n_t - n_o - gamma of a row with L1 sum s changes by at
    most 4 |dA|_1 / s (n = A/s, and both a and s move by at most |dA|_1), so
    margin < 4 |dA|_1 / s cannot be decided from A to that accuracy."""
    S_gpu = np.asarray(S_gpu)
    low = margin64 < MARGIN
    by_row = np.zeros_like(low)
    if A64 is not None and A_gpu is not None:
        A_gpu = np.asarray(A_gpu, np.float64)
        s = np.abs(A64).sum(axis=1)
        d = np.abs(A_gpu - A64).sum(axis=1)
        reld = np.where(s > 0, d / np.maximum(s, 1e-300), 0.0)
        by_row = ~low & (margin64 < 4.0 * reld[None, :])
    mism = S_gpu != S64
    seen = (np.abs(A64).sum(axis=1) > 0)[None, :] if A64 is not None else np.ones_like(low)
    st = dict(entries=int(S64.size), entries_of_seen_rows=int((seen & np.ones_like(low)).sum()),
              excluded_low_margin_seen_rows=int((low & seen).sum()),
              excluded_low_margin=int(low.sum()),
              mismatches_low_margin=int((mism & low).sum()),
              excused_by_row_difference=int((mism & by_row).sum()),
              mismatches=int((mism & ~low & ~by_row).sum()))
    return st


def assert_labels(S_gpu, S64, margin64, A64=None, A_gpu=None, what=""):
    st = compare_labels(S_gpu, S64, margin64, A64, A_gpu)
    log(f"[label parity{(' ' + what) if what else ''}] {st}")
    assert st["mismatches"] == 0, st
    return st
