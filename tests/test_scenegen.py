"""Scene cache of the input generator (CPU): a saved and reloaded batch equals
the generated one, array for array."""
import dataclasses

import numpy as np

import scenegen as sg


def test_saved_scenes_load_back_identical(tmp_path):
    a = [sg.make_config("C1", n=300, views=2, res=32), sg.make_config("C1", seed=4, n=500, views=3, res=40)]
    a[1].E = 5
    path = str(tmp_path / "s.npz")
    sg.save_scenes(path, a)
    b = sg.load_scenes(path)
    assert len(b) == 2
    for x, y in zip(a, b):
        for f in dataclasses.fields(x):
            u, v = getattr(x, f.name), getattr(y, f.name)
            if f.name == "masks":
                assert len(u) == len(v)
                assert all(np.array_equal(m1, m2) and m1.dtype == m2.dtype for m1, m2 in zip(u, v))
            elif isinstance(u, np.ndarray):
                assert np.array_equal(u, v) and u.dtype == v.dtype, f.name
            else:
                assert u == v, f.name
