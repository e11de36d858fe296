"""Pins of the oracle's per-Gaussian diagnostics (supplement "Scene
segmentation extension"; Sec. 4.8 fewer masks), CPU only: hand-counted rows,
the generator's ground-truth labels, and invariants of the assignment."""
import numpy as np

import oracle as O
import scenegen as sg


def test_hand_counted_rows():
    A = np.array([[0.0, 0.0, 0.0],      # unseen: 0 objects
                  [1.0, 0.0, 0.0],      # 1
                  [1.0, 2.0, 3.0],      # 3 (2 at rel_eps 0.2: 1 <= 0.2 * 6)
                  [0.0, 5.0, 5.0],      # 2
                  [0.1, 0.1, 9.8]])     # 3 (1 at rel_eps 0.2)
    c, m, o = O.diagnose64(A)
    assert c.tolist() == [1, 1, 1, 2] and m is None and o is None
    c, _, _ = O.diagnose64(A, rel_eps=0.2)
    assert c.tolist() == [1, 2, 2, 0]
    S = np.array([[1, 0, 0, 0, 0], [0, 1, 1, 0, 0], [0, 1, 0, 0, 1]], np.uint8)
    gt = np.array([0, 1, 2, 2, 7])
    _, m, o = O.diagnose64(None, S, gt)
    assert m.tolist() == [1, 3, 1, 0]
    assert o.tolist() == [[1, 1, 1], [1, 2, 1], [0, 2, 2]]
    assert np.allclose(O.iou_of(o), [1.0, 0.5, 0.0])


def test_exact_labels_give_iou_one_and_one_member_each():
    sc = sg.make_config("C1")
    gt = sc.gt
    S = np.stack([(gt == e) for e in range(sc.E)]).astype(np.uint8)
    _, m, o = O.diagnose64(None, S, gt)
    assert np.all(O.iou_of(o) == 1.0)
    assert m.tolist() == [0, sc.n, 0]


def test_diagnostics_of_a_solved_scene():
    sc = sg.make_config("C1")
    ref = O.solve64(sc, O.params())
    A = ref["A"]
    n, E = A.shape
    for gamma in (-0.5, -0.2, 0.0, 0.3):
        S, _ = O.assign64(A, gamma)
        c, m, o = O.diagnose64(A, S, sc.gt)
        assert int(c.sum()) == n and int(m.sum()) == n
        # the subsets are exclusive for a non-negative bias (Sec. 3.3)
        if gamma >= 0:
            assert int(m[2:].sum()) == 0
        # for a bias above -1 a Gaussian joins only objects it contributes to,
        # so no more Gaussians hold >= j memberships than >= j contributions
        for j in range(1, E + 1):
            assert int(m[j:].sum()) <= int(c[j:].sum())
        # the ray-cast masks follow the generator's labels: every object keeps
        # nearly all of its own Gaussians (recall), whatever it adds at its surface
        if gamma == 0.0:
            recall = o[:, 0].astype(float) / o[:, 2]
            assert np.all(recall > 0.9)
    # unseen Gaussians sit in bin 0 of the contribution count
    unseen = int(np.sum(A.sum(1) == 0))
    c, _, _ = O.diagnose64(A)
    assert int(c[0]) == unseen
