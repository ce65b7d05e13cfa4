"""Pins of the partitioned oracle (oracle.partitioned): its ranges, read in
key order, rebuild numpy's sort of the whole input exactly, with each range
at the offset its key counts fix, for every width, for inputs that force
splits down to single key values, and for one-value inputs."""
import numpy as np
import pytest

import fsgen
from oracle.partitioned import partitioned_sort, plan_ranges


def rebuild(keys, bits, cap, threads=3, chunk=1 << 12):
    parts, expect_off = [], 0
    for off, exp in partitioned_sort(keys, bits, cap, chunk=chunk, threads=threads):
        assert off == expect_off
        assert exp.size <= cap or (exp.size and np.all(exp == exp[0]))
        parts.append(np.asarray(exp))
        expect_off += exp.size
    assert expect_off == keys.size
    return np.concatenate(parts) if parts else np.empty(0, dtype=keys.dtype)


@pytest.mark.parametrize("bits", [16, 32, 64])
@pytest.mark.parametrize("dist", ["uniform", "small20", "hot90", "equal"])
def test_ranges_rebuild_the_sorted_array(bits, dist):
    if dist not in fsgen.valid_dists(bits):
        pytest.skip("distribution not defined for this width")
    n = 30011
    keys = fsgen.keys_host(dist, bits, n, fsgen.seed_for(5, 1) + bits)
    for cap in (n, 4099, 257):
        got = rebuild(keys, bits, cap)
        assert np.array_equal(got, np.sort(keys, kind="stable")), (bits, dist, cap)


def test_splits_reach_single_values():
    # 64-bit keys below 2^20 share their top 44 bits: the top window's one
    # bin holds every key and is split twice before the values part
    keys = fsgen.keys_host("small20", 64, 20000, 77) & np.uint64(0xF)  # 16 values
    plan = plan_ranges(keys, 64, 1000, chunk=1 << 10, threads=2)
    assert len(plan.tables) == 4  # bits 48-63, 32-47, 16-31, 0-15
    singles = [r for r in plan.ranges if r[1] is not None]
    assert len(singles) == 16 and sum(r[0] for r in singles) == keys.size
    assert np.array_equal(rebuild(keys, 64, 1000), np.sort(keys))


def test_empty_and_tiny():
    for n in (0, 1, 2):
        keys = np.arange(n, dtype=np.uint64)[::-1].copy()
        assert np.array_equal(rebuild(keys, 64, 1), np.sort(keys))


def test_a_dropped_key_is_caught():
    """A planted mistake (one key lost while grouping) changes the rebuilt
    array, so the pins above would catch it."""
    keys = fsgen.keys_host("uniform", 32, 5000, 3)
    good = rebuild(keys, 32, 700)
    bad = np.delete(keys, 1234)
    assert not np.array_equal(rebuild(bad, 32, 700), good)
