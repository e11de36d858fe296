"""The tuner on a small scene: every candidate's result agrees with the
defaults, the pick is the fastest valid one, and the picked settings pass the
oracle parity bar."""
import numpy as np
import pytest
import torch

import oracle as O
import scenegen as sg
from paper_2409_08270_amd import _lib as L
from paper_2409_08270_amd import tune as T
from tests._parity import assert_A, assert_labels, log

pytestmark = pytest.mark.gpu


def test_tuner_picks_a_valid_setting_that_matches_the_oracle(tmp_path):
    sc = sg.make_config("C1", n=1500, views=4, res=96)
    cands = [T.reference(),
             {"params": {"tile_w": 32, "tile_h": 8, "tile_order": 1}, "opts": {"reduction": L.FS_RED_LDS, "lanes": 1}},
             {"params": {"tile_w": 8, "tile_h": 32, "tile_order": 0},
              "opts": {"reduction": L.FS_RED_LDS2SUM, "lanes": 2}}]
    e = T.tune(sc, cands, steps=2, warmup=1, min_gain=0.0, log=log)
    rows = e["candidates"]
    assert len(rows) == 3 and T._same(rows[0], T.reference())
    # the support is an ellipse, so tile shape and work order change A only by summation order
    assert all(r["valid"] for r in rows), rows
    assert e["ms"] == min(r["ms"] for r in rows)
    path = str(tmp_path / "t.json")
    table = T.load(path)
    table["entries"][T.scene_key(sc)] = e
    T.save(table, path)
    pick = T.lookup(T.load(path), T.scene_key(sc))
    assert pick == {"params": e["params"], "opts": e["opts"]}
    # the picked settings against the oracle
    ctx = L.Context()
    ds = L.DeviceScene(sc)
    b = L.Batch(ctx, [ds], L.params(**pick["params"]), gammas=[0.0], **pick["opts"])
    b.run()
    torch.cuda.synchronize()
    ctx.status(raise_on_error=True)
    A = b.A_hi[0].double()
    if b.A_lo[0] is not None:
        A = A + b.A_lo[0].double()
    prm = pick["params"]
    ref = O.solve64(sc, O.params(tile_w=prm["tile_w"], tile_h=prm["tile_h"]))
    A = A.cpu().numpy()
    assert_A(A, ref["A"], ref["slack"], what="tuned settings")
    S64, m64 = O.assign64(ref["A"], 0.0)
    assert_labels(b.S[0].cpu().numpy(), S64, m64, ref["A"], A, what="tuned settings")
    b.close()
