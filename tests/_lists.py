"""Bit-exact comparison of the batched solve's own tile lists (read back per
chunk through fs_batch_chunk_lists) with the oracle's binning (tests only)."""
import numpy as np

import oracle as O
from paper_2409_08270_amd.solve import tiles_of


def check_chunk_lists(batch, scenes, want, prm, what=""):
    """For every (scene, view) in `want`, the view's ids and per-tile ranges in
    the chunk that holds it equal O.bin_view's, entry for entry. Returns
    (entries compared, chunks visited, packed chunks seen)."""
    want = set((int(s), int(v)) for s, v in want)
    oprm = O.params(tile_w=prm.tile_w, tile_h=prm.tile_h, sigma_k=prm.sigma_k, lowpass=prm.lowpass,
                    znear=prm.znear, guard=prm.guard, alpha_min=prm.alpha_min, alpha_max=prm.alpha_max,
                    t_min=prm.t_min, fp64_cond=prm.fp64_cond)
    checked, chunks, packed = 0, 0, set()
    found = set()
    for c in range(batch.info()["n_chunks"]):
        inf, vals, ranges, refs = batch.chunk_lists(c)
        chunks += 1
        tbase = 0
        off_expected = 0
        for si, v in refs:
            sc = scenes[si]
            T = tiles_of(int(sc.W[v]), int(sc.H[v]), prm)
            r = ranges[tbase:tbase + T].astype(np.int64)
            nz = r[:, 1] > r[:, 0]
            # the views' lists are consecutive in the chunk, in chunk order
            if nz.any():
                assert r[nz, 0].min() == off_expected, (what, c, si, v)
                off_expected = int(r[nz, 1].max())
            assert np.all(r[~nz] == 0), (what, c, si, v)
            if (si, v) in want:
                b = O.bin_view(sc, v, oprm)
                ro = b["ranges"].astype(np.int64)
                on = ro[:, 1] > ro[:, 0]
                assert np.array_equal(nz, on), (what, c, si, v, "non-empty tiles differ")
                assert np.array_equal(r[:, 1] - r[:, 0], ro[:, 1] - ro[:, 0]), (what, c, si, v, "list lengths")
                if on.any():
                    lo = int(r[nz, 0].min())
                    hi = int(r[nz, 1].max())
                    assert np.array_equal(vals[lo:hi], b["g"]), (what, c, si, v, "list entries")
                    assert np.array_equal(r[on] - lo, ro[on]), (what, c, si, v, "ranges")
                checked += int(b["g"].size)
                found.add((si, v))
                if inf["packed"]:
                    packed.add(c)
            tbase += T
        assert tbase == inf["n_tiles"], (what, c)
        assert off_expected == inf["n_pairs"], (what, c, off_expected, inf["n_pairs"])
    assert found == want, (what, sorted(want - found))
    return checked, chunks, len(packed)
