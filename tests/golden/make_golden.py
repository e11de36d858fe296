"""Writes the oracle snapshots in this folder (calls only oracle/ and the
seeded input generator). Run from the repository root:

    python tests/golden/make_golden.py

The paper prints no numeric worked example (its tables need its datasets), so
the fixtures here are regression snapshots of the pinned oracle on tiny seeded
scenes, plus a hand-derived closed-form case. A change to a snapshot must come
with a change to the oracle's arithmetic whose commit message names the
passage of the paper that justifies it.
"""
import json
import math
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle as O  # noqa: E402
import scenegen as sg  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
CASES = [dict(seed=s, n=10, views=3, res=32, E=e, masks=m)
         for s, e, m in ((0, 2, "random"), (1, 2, "raycast"), (2, 3, "random"))]


def snapshot(case):
    sc = sg.make_tiny(**case)
    ref = O.solve64(sc, O.params(**O.EXACT))
    out = {"case": case, "params": "exact preset (alpha_min=0, alpha_max=1, t_min=0)",
           "A": ref["A"].tolist(), "blends": int(ref["blends"])}
    for gamma in (0.0, 0.3, -0.3):
        S, m = O.assign64(ref["A"], gamma)
        out[f"S_gamma_{gamma:+.1f}"] = S.tolist()
    return out


def main():
    snaps = [snapshot(c) for c in CASES]
    with open(os.path.join(HERE, "tiny_oracle.json"), "w") as f:
        json.dump({"source": "oracle/ on scenegen.make_tiny scenes; see make_golden.py",
                   "cases": snaps}, f, indent=1)
    print(f"wrote {len(snaps)} snapshots")


if __name__ == "__main__":
    main()
