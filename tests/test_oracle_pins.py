"""Pins of the CPU oracle to things other than itself (no GPU needed).

Each pin checks the oracle against something the paper or plain
mathematics fixes -- brute force over tiny inputs, Python's sorted() on
(key, index), numpy's stable argsort and bincount, closed forms of the
presorted / reverse / all-equal inputs -- and the planted-mistake test
rebuilds the oracle with a deliberate bug and checks that some pin fails.
"""
import itertools
import os
import tempfile

import numpy as np
import pytest

import oracle
from oracle import build as oracle_build
from tests.checks import check_index_pairs, check_keys

DT = {1: np.uint8, 2: np.uint16, 4: np.uint32, 8: np.uint64}
WIDTHS = (1, 2, 4, 8)


def _brute_sort(keys):
    """Python sorted() on (key, original index): the definition of a stable
    ascending sort."""
    order = sorted(range(len(keys)), key=lambda i: (int(keys[i]), i))
    return [int(keys[i]) for i in order], order


# ----------------------------------------------------------------- pin bodies
# Each takes a loaded oracle library so the planted-mistake test can run the
# same pins against a deliberately broken build.

def _alphabets(kb):
    """Key alphabets that differ in the lowest, a middle and the top digit."""
    p = 8 * kb
    if kb == 1:
        return [[0, 1, 0x80, 0xFF], [0x0F, 0x10, 0x7F, 0x81]]
    return [
        [0, 1, 1 << (p - 8), (1 << p) - 1],
        [0x0100, 0x00FF, 1 << (p // 2), (1 << (p - 1)) | 1],
    ]


def _wide_payload(n):
    """n distinct 8-byte payloads whose upper 4 bytes all differ and whose
    lower 4 bytes repeat, so that a payload moved with only its low half
    (or a 4-byte stride) comes out wrong."""
    i = np.arange(n, dtype=np.uint64)
    return ((i + np.uint64(1)) << np.uint64(36)) | (i % np.uint64(3))


def pin_exhaustive_tiny(lib):
    """Every sequence of length <= 4 over alphabets that differ in the
    lowest, a middle and the top digit, for 8/16/32/64-bit keys, with
    4-byte index payloads and with 8-byte payloads above 2^32."""
    for kb in WIDTHS:
        for alpha in _alphabets(kb):
            for length in range(0, 5):
                for seq in itertools.product(alpha, repeat=length):
                    keys = np.array(seq, dtype=DT[kb])
                    idx = np.arange(length, dtype=np.uint32)
                    ko, vo = oracle.sort(keys, idx, lib=lib)
                    exp_k, exp_v = _brute_sort(keys)
                    assert ko.tolist() == exp_k, (kb, seq)
                    assert vo.tolist() == exp_v, (kb, seq)
                    wide = _wide_payload(length)
                    ko8, vo8 = oracle.sort(keys, wide, lib=lib)
                    assert ko8.tolist() == exp_k, (kb, seq)
                    assert vo8.tolist() == [int(wide[i]) for i in exp_v], (kb, seq)
                    assert oracle.sort(keys, lib=lib).tolist() == exp_k, (kb, seq)


def pin_random_vs_numpy(lib):
    """Random keys (with heavy duplication) against numpy's stable argsort,
    with 4-byte index payloads and 8-byte payloads above 2^32."""
    rng = np.random.default_rng(1234)
    for kb in WIDTHS:
        info = np.iinfo(DT[kb])
        for n in (1, 2, 3, 17, 255, 256, 257, 1000, 4099):
            for spread in ("full", "few"):
                if spread == "full":
                    keys = rng.integers(0, int(info.max), size=n, dtype=DT[kb], endpoint=True)
                else:
                    pool = rng.integers(0, int(info.max), size=5, dtype=DT[kb], endpoint=True)
                    keys = pool[rng.integers(0, 5, size=n)]
                idx = np.arange(n, dtype=np.uint32)
                ko, vo = oracle.sort(keys, idx, lib=lib)
                order = np.argsort(keys, kind="stable")
                assert np.array_equal(ko, keys[order]), (kb, n, spread)
                assert np.array_equal(vo, order.astype(np.uint32)), (kb, n, spread)
                assert np.array_equal(oracle.sort(keys, lib=lib), keys[order])
                wide = _wide_payload(n) ^ rng.integers(0, 1 << 32, size=n, dtype=np.uint64)
                ko8, vo8 = oracle.sort(keys, wide, lib=lib)
                assert np.array_equal(ko8, keys[order]), (kb, n, spread)
                assert np.array_equal(vo8, wide[order]), (kb, n, spread)


def pin_closed_forms(lib):
    """All-equal and presorted inputs sort to the identity permutation;
    reverse-sorted input comes out as its blocks in reverse order, each block
    in input order (the closed forms of the presorted and reverse recipes)."""
    for n in (1, 5, 300, 70000):
        idx = np.arange(n, dtype=np.uint32)
        for kb in WIDTHS:
            eq = np.full(n, 0xBEEF if kb > 1 else 0xBE, dtype=DT[kb])
            ko, vo = oracle.sort(eq, idx, lib=lib)
            assert np.array_equal(vo, idx) and np.array_equal(ko, eq)
        pre = ((np.arange(n, dtype=np.uint64) << np.uint64(16)) // np.uint64(n)).astype(np.uint16)
        ko, vo = oracle.sort(pre, idx, lib=lib)
        assert np.array_equal(vo, idx) and np.array_equal(ko, pre)
        rev = (65535 - pre.astype(np.int64)).astype(np.uint16)
        ko, vo = oracle.sort(rev, idx, lib=lib)
        # blocks of equal keys: [s_j, e_j) in input order
        starts = [0] + [i for i in range(1, n) if rev[i] != rev[i - 1]]
        ends = starts[1:] + [n]
        expect = np.concatenate([np.arange(s, e) for s, e in reversed(list(zip(starts, ends)))])
        assert np.array_equal(vo, expect.astype(np.uint32))
        assert np.array_equal(ko, rev[::-1])


def pin_histogram(lib):
    """Leaf counters equal numpy.bincount of the digit, for several digit
    positions and widths."""
    rng = np.random.default_rng(7)
    for kb in WIDTHS:
        keys = rng.integers(0, int(np.iinfo(DT[kb]).max), size=5000, dtype=DT[kb], endpoint=True)
        keys[:700] = keys[0]  # a heavy bin
        p = 8 * kb
        shapes = ((0, 8), (3, 5), (1, 7)) if kb == 1 else ((0, 8), (8, 8), (p - 8, 8), (0, 16), (p - 16, 16), (3, 5))
        for shift, bits in shapes:
            h = oracle.histogram(keys, shift, bits, lib=lib)
            d = ((keys.astype(np.uint64) >> np.uint64(shift)) & np.uint64((1 << bits) - 1)).astype(np.int64)
            assert np.array_equal(h, np.bincount(d, minlength=1 << bits).astype(np.uint64)), (kb, shift, bits)


def pin_rank_and_select(lib):
    """GetIndex (exclusive prefix) equals the brute-force count of smaller
    keys; GetItem(i) equals the i-th smallest key; the expansion of the full
    histogram equals the sorted keys."""
    rng = np.random.default_rng(99)
    for n in (0, 1, 9, 40):
        keys = rng.integers(0, 16, size=n).astype(np.uint16)
        h = oracle.histogram(keys, 0, 4, lib=lib)
        pre = oracle.exclusive_scan(h, lib=lib)
        for v in range(16):
            assert int(pre[v]) == sum(1 for k in keys if k < v), (n, v)
        assert int(pre[16]) == n
        srt = sorted(int(k) for k in keys)
        for i in range(n):
            assert oracle.select(h, i, lib=lib) == srt[i]
        assert oracle.select(h, n, lib=lib) == 16
        assert oracle.expand(h, np.uint16, lib=lib).tolist() == srt
    # a 16-bit histogram expands to the sorted keys of a larger input
    keys = rng.integers(0, 65536, size=20000).astype(np.uint16)
    h = oracle.histogram(keys, 0, 16, lib=lib)
    assert np.array_equal(oracle.expand(h, np.uint16, lib=lib), np.sort(keys))


def pin_segments(lib):
    """Each segment sorts as it would alone (brute force on tiny segments)."""
    rng = np.random.default_rng(5)
    segs = [rng.integers(0, 4, size=m).astype(np.uint16) for m in (0, 1, 3, 7)]
    segs += [rng.integers(0, 2 ** 32, size=m, dtype=np.uint64).astype(np.uint32) for m in (2, 6)]
    out = oracle.sort_segments(segs, lib=lib)
    for s, o in zip(segs, out):
        assert o.tolist() == _brute_sort(s)[0]


PINS = [pin_exhaustive_tiny, pin_random_vs_numpy, pin_closed_forms, pin_histogram,
        pin_rank_and_select, pin_segments]


@pytest.mark.parametrize("pin", PINS, ids=lambda f: f.__name__)
def test_oracle_pin(pin):
    pin(oracle.load())


def test_oracle_rejects_bad_arguments():
    lib = oracle.load()
    k = np.zeros(4, dtype=np.uint16)
    assert lib.oracle_sort(k.ctypes.data, k.ctypes.data, None, None, 4, 3, 0) != 0
    assert lib.oracle_sort(k.ctypes.data, k.ctypes.data, None, None, 4, 2, 5) != 0
    assert lib.oracle_histogram(k.ctypes.data, 4, 2, 10, 8, k.ctypes.data) != 0


def test_checker_rejects_wrong_results():
    """The invariant checker must flag unsorted, unstable and
    non-permutation outputs (so a GPU parity test built on it can fail)."""
    keys = np.array([3, 1, 3, 2, 1], dtype=np.uint16)
    idx = np.arange(5, dtype=np.uint32)
    ko, vo = oracle.sort(keys, idx)
    check_index_pairs(keys, ko, vo)
    check_keys(keys, ko, 16)
    with pytest.raises(AssertionError):  # unstable: swap two equal keys' payloads
        bad = vo.copy(); bad[0], bad[1] = bad[1], bad[0]
        check_index_pairs(keys, ko, bad)
    with pytest.raises(AssertionError):  # unsorted
        check_index_pairs(keys, keys, idx)
    with pytest.raises(AssertionError):  # duplicated payload
        bad = vo.copy(); bad[0] = bad[1]
        check_index_pairs(keys, ko, bad)
    with pytest.raises(AssertionError):  # keys-only multiset changed
        check_keys(keys, np.array([1, 1, 2, 2, 3], dtype=np.uint16), 16)


PLANTS = ["ORACLE_PLANT_UNSTABLE", "ORACLE_PLANT_SKIP_TOP_DIGIT",
          "ORACLE_PLANT_HIST_OFF_BY_ONE", "ORACLE_PLANT_INCLUSIVE_SCAN",
          "ORACLE_PLANT_PAYLOAD_HALF", "ORACLE_PLANT_KEY8_READS_16"]


def _run_pins_against(path):
    """Child-process entry: run every pin against the library at `path` and
    exit non-zero when any pin fails."""
    lib = oracle.load(path)
    failed = []
    for pin in PINS:
        try:
            pin(lib)
        except AssertionError:
            failed.append(pin.__name__)
    print("FAILED_PINS", failed)
    raise SystemExit(1 if failed else 0)


@pytest.mark.parametrize("plant", PLANTS)
def test_planted_mistake_is_caught(plant):
    """Rebuild the oracle with one deliberate mistake; at least one pin must
    fail against it.  The pins run in a child process, because a planted
    mistake may also corrupt memory (which counts as caught)."""
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "liboracle_planted.so")
        oracle_build.build(path, defines=[plant])
        code = ("import sys; sys.path.insert(0, %r); "
                "from tests.test_oracle_pins import _run_pins_against; "
                "_run_pins_against(%r)" % (root, path))
        r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True,
                           timeout=600)
        assert r.returncode != 0, f"no pin caught {plant}: {r.stdout[-500:]}"


@pytest.mark.parametrize("key_bytes,val_bytes", [(1, 8), (2, 0), (2, 4), (4, 4), (8, 0), (8, 8)])
def test_threaded_oracle_equals_single_thread(key_bytes, val_bytes):
    """The CPU-baseline timing variant gives the same bytes as the oracle
    for any thread count, including more threads than keys."""
    rng = np.random.default_rng(key_bytes * 10 + val_bytes)
    kdt = DT[key_bytes]
    for n in (0, 1, 5, 1000, 70_001):
        k = rng.integers(0, 1 << 63, size=n, dtype=np.uint64).astype(kdt)
        k[: n // 4] = k[n // 4: 2 * (n // 4)]
        v = np.arange(n, dtype={4: np.uint32, 8: np.uint64}[val_bytes]) if val_bytes else None
        want = oracle.sort(k, v)
        for threads in (1, 3, 8, 64):
            got = oracle.sort_mt(k, v, threads=threads)
            if v is None:
                assert np.array_equal(got, want), (n, threads)
            else:
                assert np.array_equal(got[0], want[0]) and np.array_equal(got[1], want[1]), (n, threads)
