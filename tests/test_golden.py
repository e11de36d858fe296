"""The oracle reproduces its stored snapshots (tests/golden/tiny_oracle.json,
written by tests/golden/make_golden.py from oracle/ only)."""
import json
import os

import numpy as np

import oracle as O
import scenegen as sg

HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def test_oracle_matches_its_snapshots():
    data = json.load(open(os.path.join(HERE, "tiny_oracle.json")))
    assert len(data["cases"]) == 3
    for snap in data["cases"]:
        sc = sg.make_tiny(**snap["case"])
        ref = O.solve64(sc, O.params(**O.EXACT))
        A0 = np.array(snap["A"])
        assert ref["A"].shape == A0.shape
        assert np.allclose(ref["A"], A0, rtol=1e-12, atol=1e-15)
        assert int(ref["blends"]) == snap["blends"]
        for gamma in (0.0, 0.3, -0.3):
            S, _ = O.assign64(ref["A"], gamma)
            assert np.array_equal(S, np.array(snap[f"S_gamma_{gamma:+.1f}"], dtype=np.uint8))
