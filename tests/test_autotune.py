"""Host logic of the segmented-sort autotuner and the tuning table of the
C-ABI library (no GPU: setting and reading the table makes no device call)."""
import ctypes
import math
import os

import pytest

from paper_2605_10390_amd import autotune as at

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2605_10390_amd", "libfsort.so")

FIELDS = [n for e in at.ORDER for n in (e if isinstance(e, tuple) else (e,))]

START = {"small_max_keys": [at.NEVER, at.NEVER, at.NEVER], "expand16_min_keys": 8192,
         "expand16_split_keys": 1 << 18, "expand16_wgs_per_cu": 1, "large_wg_max_keys": 0, "tile_items": 16,
         "tile_threads": 256, "large_wgs_per_cu": 2, "small_wgs_per_cu": 2}


def separable_cost(target):
    """A cost with a unique minimum at `target`: 10 ms plus a penalty per
    field that grows with the candidate-list distance from the target."""
    def cost(t):
        ms = 10.0
        for name in FIELDS:
            cand = at.CANDIDATES[name]
            ms += 0.5 * abs(cand.index(at.get_field(t, name)) - cand.index(at.get_field(target, name)))
        return ms
    return cost


def test_search_finds_separable_optimum():
    target = at.with_field(at.with_field(at.with_field(START, "expand16_min_keys", 2048),
                                         "large_wgs_per_cu", 6), "small_max_keys.1", 1024)
    target = at.with_field(target, "tile_items", 8)
    best, ms, hist = at.coordinate_search(separable_cost(target), START)
    assert best == target
    assert ms == pytest.approx(10.0)


def test_search_caches_and_counts():
    calls = []

    def cost(t):
        calls.append(at.key_of(t))
        return separable_cost(START)(t)

    best, ms, hist = at.coordinate_search(cost, START, sweeps=3)
    assert best == START  # already optimal: nothing moves, one sweep is enough
    assert len(calls) == len(set(calls)) == len(hist)
    per_entry = [math.prod(len(at.CANDIDATES[n]) for n in (e if isinstance(e, tuple) else (e,))) - 1
                 for e in at.ORDER]
    assert len(hist) == 1 + sum(per_entry)


def test_grouped_fields_find_a_joint_optimum():
    """A cost where the tile size only pays with many workgroups: one field
    at a time would stay at the start, the grouped search finds the pair."""
    def cost(t):
        if t["tile_items"] == 8 and t["large_wgs_per_cu"] == 6:
            return 5.0
        if t["tile_items"] == 8:
            return 12.0
        return 10.0

    best, ms, _ = at.coordinate_search(cost, START)
    assert (best["tile_items"], best["large_wgs_per_cu"]) == (8, 6) and ms == 5.0


def test_margin_ignores_noise():
    # every other tuning is 0.5% faster: below the 1% margin, so the start stays
    def cost(t):
        return 10.0 if t == START else 9.95

    best, ms, _ = at.coordinate_search(cost, START, margin=0.01)
    assert best == START and ms == 10.0


def test_search_moves_only_on_improvement():
    # a cost where only tile_items matters, 8 is 20% faster
    def cost(t):
        return 8.0 if t["tile_items"] == 8 else 10.0

    best, ms, _ = at.coordinate_search(cost, START)
    assert best["tile_items"] == 8 and ms == 8.0
    assert {k: v for k, v in best.items() if k != "tile_items"} == \
        {k: v for k, v in START.items() if k != "tile_items"}


@pytest.mark.skipif(not os.path.exists(LIB), reason="libfsort.so not built")
def test_library_accepts_every_candidate_and_rejects_out_of_range():
    import paper_2605_10390_amd as fs
    d = fs.default_tuning().as_dict()
    try:
        for name in FIELDS:
            for v in at.CANDIDATES[name]:
                t = at.with_field(d, name, v)
                fs.set_tuning(fs.SegTuning.from_dict(t))
                assert fs.get_tuning().as_dict() == t
        for name, v in (("tile_items", 12), ("tile_items", 32), ("large_wgs_per_cu", 0),
                        ("large_wgs_per_cu", 9), ("small_wgs_per_cu", 0), ("small_wgs_per_cu", 5),
                        ("expand16_wgs_per_cu", 0), ("expand16_wgs_per_cu", 3), ("tile_threads", 128),
                        ("tile_threads", 1024)):
            before = fs.get_tuning().as_dict()
            with pytest.raises(fs.FsError):
                fs.set_tuning(fs.SegTuning.from_dict(at.with_field(d, name, v)))
            assert fs.get_tuning().as_dict() == before
        fs.set_tuning(None)
        assert fs.get_tuning().as_dict() == d
    finally:
        fs.set_tuning(None)


@pytest.mark.skipif(not os.path.exists(LIB), reason="libfsort.so not built")
def test_tuned_call_checks_tuning_before_anything():
    import paper_2605_10390_amd as fs
    L = fs.lib()
    bad = fs.default_tuning()
    bad.tile_items = 3
    size = ctypes.c_size_t(0)
    st = L.fs_sort_segmented_tuned(None, 10, 1000, 100, 0, ctypes.byref(bad), None, ctypes.byref(size), None)
    assert st == fs.FS_ERR_INVALID_ARG
    good = fs.default_tuning()
    st = L.fs_sort_segmented_tuned(None, 10, 1000, 100, 0, ctypes.byref(good), None, ctypes.byref(size), None)
    assert st == 0 and size.value > 0


def test_save_load_roundtrip(tmp_path):
    if not os.path.exists(LIB):
        pytest.skip("libfsort.so not built")
    import paper_2605_10390_amd as fs
    t = fs.SegTuning.from_dict(at.with_field(START, "large_wgs_per_cu", 4))
    p = tmp_path / "t.json"
    at.save(str(p), t, {"best_ms": 1.0})
    assert at.load(str(p)).as_dict() == t.as_dict()
