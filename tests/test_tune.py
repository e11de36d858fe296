"""Tuning table: keys, candidate settings and table I/O (CPU)."""
import json

from paper_2409_08270_amd import _lib as L
from paper_2409_08270_amd import tune as T


def test_workload_key_buckets_the_gaussian_count():
    assert T.workload_key(200000, 640, 480, 2, 50) == "E2-640x480-N262144-V50"
    assert T.workload_key(131072, 640, 480, 2, 50) == "E2-640x480-N131072-V50"
    assert T.workload_key(131073, 640, 480, 2, 50) == "E2-640x480-N262144-V50"


def test_candidates_cover_the_tunable_settings_and_include_the_defaults():
    cs = T.candidates(640, 480)
    shapes = {(c["params"]["tile_w"], c["params"]["tile_h"]) for c in cs}
    assert shapes == {(16, 16), (32, 8), (8, 32)}
    assert all(c["params"]["tile_w"] * c["params"]["tile_h"] == 256 for c in cs)
    assert {c["opts"]["reduction"] for c in cs} == {L.FS_RED_LDS2SUM, L.FS_RED_DET}
    assert {c["opts"]["reduction"] for c in T.candidates(640, 480, compensated=False)} == {
        L.FS_RED_LDS, L.FS_RED_LDS2SUM, L.FS_RED_DET}
    assert {c["opts"]["lanes"] for c in cs} == {1, 2, 3, 4}
    assert {c["params"]["tile_order"] for c in cs} == {0, 1}
    assert {c["params"]["persistent"] for c in cs} == {0, 1}
    assert {c["params"]["lds_batch"] for c in cs} == {64, 128, 256}
    assert {c["opts"]["depth_slabs"] for c in cs} == {1, 2, 3}
    assert len(cs) == 3 * 2 * 4 * 2 * 3 * 3 * 2
    assert sum(T._same(c, T.reference()) for c in cs) == 1
    # the reference is what the library's defaults are
    p = L.params()
    assert T.reference()["params"] == {"tile_w": p.tile_w, "tile_h": p.tile_h, "tile_order": p.tile_order,
                                       "persistent": p.persistent, "lds_batch": p.lds_batch or 256}
    o = L.batch_opts()
    assert o.lanes == 0 and o.reduction == L.FS_RED_AUTO  # 0: two lanes; auto: LDS + two-sum with A_lo
    assert o.depth_slabs == 0  # 0: one slab


def test_batch_key_names_single_scenes_like_scene_key():
    import scenegen as sg
    sc = sg.make_config("C1", n=300, views=2, res=32)
    assert T.batch_key([sc]) == T.scene_key(sc)
    sc2 = sg.make_config("C1", seed=3, n=500, views=3, res=48)
    k = T.batch_key([sc, sc2])
    assert k == f"B2-N1024-P{T._bucket(2 * 32 * 32 + 3 * 48 * 48)}-V5-E2"


def test_table_round_trip(tmp_path):
    path = str(tmp_path / "t.json")
    t = T.load(path)
    assert t == {"version": 1, "entries": {}}
    t["entries"]["E2-64x64-N1024-V3"] = {"params": {"tile_w": 32, "tile_h": 8, "tile_order": 1},
                                        "opts": {"reduction": L.FS_RED_LDS, "lanes": 1}, "ms": 1.0,
                                        "reference_ms": 1.2, "candidates": []}
    T.save(t, path)
    back = T.load(path)
    assert back == json.loads(json.dumps(t))
    hit = T.lookup(back, "E2-64x64-N1024-V3")
    assert hit == {"params": {"tile_w": 32, "tile_h": 8, "tile_order": 1},
                   "opts": {"reduction": L.FS_RED_LDS, "lanes": 1}}
    assert T.lookup(back, "E3-64x64-N1024-V3") is None


def test_committed_table_is_well_formed():
    t = T.load()
    for key, e in t["entries"].items():
        assert key[0] in "EB" and "-N" in key
        assert e["params"]["tile_w"] * e["params"]["tile_h"] == 256
        assert e["opts"]["reduction"] in (L.FS_RED_LDS, L.FS_RED_LDS2SUM)
        assert 1 <= e["opts"]["lanes"] <= 4
        chosen = [c for c in e["candidates"] if T._same(c, e)]
        assert chosen and chosen[0]["valid"]
