"""Pins of the oracle's bias sweep and object extraction/removal (CPU only)."""
import numpy as np

import oracle as O


def _random_A(seed, n=300, E=5):
    rng = np.random.default_rng(seed)
    A = rng.gamma(0.5, 1.0, size=(n, E))
    A[rng.random((n, E)) < 0.3] = 0.0
    A[:7] = 0.0  # unseen Gaussians
    return A


def test_sweep_counts_shrink_as_the_bias_grows():
    # a larger bias toward "others" can only remove members (Sec. 3.2)
    A = _random_A(0)
    gammas = np.linspace(-1.0, 1.0, 21)
    S, counts = O.sweep64(A, gammas)
    assert S.shape == (21, 5, 300) and counts.shape == (21, 5)
    assert np.all(np.diff(counts, axis=0) <= 0)
    assert np.all(np.diff(S.astype(int), axis=0) <= 0)  # membership is monotone entry by entry


def test_sweep_at_the_extremes():
    A = _random_A(1)
    S, counts = O.sweep64(A, [-1.0, 1.0])
    seen = A.sum(1) > 0
    # gamma = 1: a_n > o_n + 1 is impossible since a_n <= 1
    assert counts[1].sum() == 0
    # gamma = -1: every object is taken unless all of the row's weight is on the others
    for t in range(A.shape[1]):
        others_only = seen & (A[:, t] == 0)
        assert np.array_equal(S[0, t].astype(bool), ~others_only)


def test_sweep_exclusive_for_nonnegative_bias():
    A = _random_A(2)
    S, _ = O.sweep64(A, [0.0, 0.1, 0.5])
    assert np.all(S.sum(axis=1) <= 1)


def test_extraction_and_removal_partition_the_scene():
    rng = np.random.default_rng(3)
    n = 97
    arrays = [rng.normal(size=n).astype(np.float32) for _ in range(11)]
    sel = (rng.random(n) < 0.4).astype(np.uint8)
    keep, ik = O.compact64(arrays, sel, True)
    drop, idr = O.compact64(arrays, sel, False)
    assert len(ik) + len(idr) == n and len(np.intersect1d(ik, idr)) == 0
    assert np.all(np.diff(ik) > 0) and np.all(np.diff(idr) > 0)  # original order kept
    # brute force: walk the rows
    want = [i for i in range(n) if sel[i]]
    assert list(ik) == want
    for a, k in zip(arrays, keep):
        assert np.array_equal(k, np.array([a[i] for i in want], np.float32))
    # nothing selected / everything selected
    none, i0 = O.compact64(arrays, np.zeros(n, np.uint8), True)
    assert i0.size == 0 and all(a.size == 0 for a in none)
