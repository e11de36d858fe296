"""Pins of the oracle's closed-form assignment (CPU only).

The closed form (Eq. (7); Eq. (8) per object; L1 normalisation and the
background bias of Sec. 3.2) is checked against an exhaustive search over
every labelling of Eq. (2) on tiny scenes, against an independent PyTorch
formulation built from library routines (L1 normalize, argmax with
first-index ties), and against consequences the paper states (subsets overlap
only for negative bias; the binary case is the plain majority vote).
"""
import numpy as np
import pytest
import torch
import torch.nn.functional as F

import oracle as O
import scenegen as sg

PRM = O.params()


@pytest.mark.parametrize("seed,masks", [(21, "random"), (22, "raycast"), (23, "raycast"), (24, "random")])
def test_closed_form_attains_the_exhaustive_optimum_of_eq2(seed, masks):
    sc = sg.make_tiny(seed, n=12 if seed % 2 else 10, views=3, res=32, masks=masks)
    Ws = [O.weights64(sc, v, PRM) for v in range(sc.n_views)]
    best, _, vals = O.brute_force_binary(Ws, sc.masks)
    A = O.solve64(sc, PRM)["A"]
    S, margin = O.assign64(A, 0.0)
    P = S[1].astype(np.float64)
    assert O.objective_eq2(Ws, sc.masks, P) == pytest.approx(best, rel=1e-12, abs=1e-12)
    # every labelling's objective is C + sum_i P_i (A0 - A1)  (Eq. (6))
    C = sum(float(m.sum()) for m in sc.masks)
    n = sc.n
    codes = np.arange(1 << n)
    Pall = ((codes[:, None] >> np.arange(n)[None, :]) & 1).astype(np.float64)
    assert np.allclose(vals, C + Pall @ (A[:, 0] - A[:, 1]), rtol=1e-10, atol=1e-9)


def test_multi_object_closed_form_is_optimal_per_object():
    # scene segmentation: for object t, S[t] minimises Eq. (2) against the
    # binary mask 1(M == t) (Eq. (8) with A_0 = A_others)
    sc = sg.make_tiny(31, n=10, views=3, res=32, E=4, masks="random")
    Ws = [O.weights64(sc, v, PRM) for v in range(sc.n_views)]
    A = O.solve64(sc, PRM)["A"]
    S, _ = O.assign64(A, 0.0)
    for t in range(sc.E):
        bm = [(m == t).astype(np.uint8) for m in sc.masks]
        best, _, _ = O.brute_force_binary(Ws, bm)
        assert O.objective_eq2(Ws, bm, S[t].astype(np.float64)) == pytest.approx(best, rel=1e-12, abs=1e-12)


def _torch_assign(A, gamma):
    """Independent formulation: per object, stack (others, own), L1-normalise
    with torch's normalize (eps 1e-12), bias the first row, argmax over rows."""
    At = torch.tensor(A.T, dtype=torch.float64)  # [E, n]
    E = At.shape[0]
    out = torch.zeros_like(At, dtype=torch.uint8)
    for t in range(E):
        mask = torch.ones(E, dtype=torch.bool)
        mask[t] = False
        pair = torch.stack([At[mask].sum(dim=0), At[t]])
        pair = F.normalize(pair, p=1, dim=0)
        pair[0] += gamma
        out[t] = torch.argmax(pair, dim=0).to(torch.uint8)
    return out.numpy()


@pytest.mark.parametrize("gamma", [0.0, 0.2, 0.5, -0.4, 1.0, -1.0])
def test_matches_torch_normalize_argmax(gamma):
    rng = np.random.default_rng(5)
    A = rng.exponential(size=(3000, 6))
    A[rng.random(A.shape) < 0.3] = 0.0
    A[:50] = 0.0                           # unseen Gaussians
    A[50:100, 2] = A[50:100, 3] = 1.0      # exact ties between two objects
    A[50:100, [0, 1, 4, 5]] = 0.0
    S, _ = O.assign64(A, gamma)
    assert np.array_equal(S, _torch_assign(A, gamma))


def test_binary_is_majority_vote_and_unseen_rule():
    rng = np.random.default_rng(6)
    A = rng.exponential(size=(2000, 2))
    A[:10] = 0.0
    A[10:20, 1] = A[10:20, 0]
    S, margin = O.assign64(A, 0.0)
    assert np.array_equal(S[1], (A[:, 1] > A[:, 0]).astype(np.uint8))
    assert np.array_equal(S[0], (A[:, 0] > A[:, 1]).astype(np.uint8))
    # unseen rows: normalised pair is (0, 0); labelled iff gamma < 0
    assert np.all(S[:, :10] == 0) and np.all(margin[:, :10] == 0)
    Sn, _ = O.assign64(A, -0.1)
    assert np.all(Sn[:, :10] == 1)


def test_positive_bias_is_exclusive_and_bias_is_monotone():
    rng = np.random.default_rng(7)
    A = rng.exponential(size=(5000, 9)) * (rng.random((5000, 9)) < 0.5)
    prev = None
    for gamma in np.linspace(-1, 1, 21):
        S, _ = O.assign64(A, float(gamma))
        if gamma >= 0:
            assert S.sum(axis=0).max() <= 1   # overlaps need gamma < 0
        if prev is not None:
            assert np.all(S <= prev)          # raising gamma never adds a member
        prev = S


def test_margin_definition_on_hand_values():
    A = np.array([[3.0, 1.0], [1.0, 1.0], [0.0, 2.0]])
    S, m = O.assign64(A, 0.1)
    # row 0: object 1 has (others, own) = (3, 1)/4 -> 0.25 > 0.75 + 0.1 is false
    assert S[1, 0] == 0 and m[1, 0] == pytest.approx(abs(0.25 - 0.75 - 0.1))
    # row 1: tie (0.5, 0.5): bias decides for "others"
    assert S[1, 1] == 0 and S[0, 1] == 0 and m[0, 1] == pytest.approx(0.1)
    # row 2: all weight on object 1
    assert S[1, 2] == 1 and m[1, 2] == pytest.approx(0.9) and S[0, 2] == 0
