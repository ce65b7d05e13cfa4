"""Pins of oracle.sort_ordered (signed, floating-point and descending key
orders) against things other than itself: a hand-ordered list of IEEE 754
special values in the standard's totalOrder (IEEE 754-2008, Sec. 5.10),
Python's own stable `sorted` (also with reverse=True, which keeps equal
elements in input order), numpy's float sort on finite values, and the C
counting-sort oracle for unsigned keys."""
import numpy as np
import pytest

import oracle

# binary32 bit patterns in totalOrder: negative NaNs (quiet above
# signalling, larger payload first), -inf, negative numbers, -0, +0,
# positive numbers, +inf, positive NaNs (signalling first, smaller payload
# first)
TOTAL_ORDER_F32 = [
    0xFFFFFFFF, 0xFFC00001, 0xFFC00000, 0xFFBFFFFF, 0xFF800001,  # -NaN
    0xFF800000,                                                  # -inf
    0xFF7FFFFF, 0xC0000000, 0xBF800000, 0x80800000,              # -max .. -min normal
    0x807FFFFF, 0x80000001,                                      # negative subnormals
    0x80000000, 0x00000000,                                      # -0, +0
    0x00000001, 0x007FFFFF, 0x00800000, 0x3F800000, 0x7F7FFFFF,  # +subnormals .. +max
    0x7F800000,                                                  # +inf
    0x7F800001, 0x7FBFFFFF, 0x7FC00000, 0x7FC00001, 0x7FFFFFFF,  # +NaN
]
TOTAL_ORDER_F16 = [0xFFFF, 0xFE00, 0xFC01, 0xFC00, 0xFBFF, 0xBC00, 0x8001, 0x8000,
                   0x0000, 0x0001, 0x3C00, 0x7BFF, 0x7C00, 0x7C01, 0x7E00, 0x7FFF]


def _widen_f32_to_f64(bits32):
    """The same classes in binary64: sign, exponent all-ones or rebiased,
    mantissa moved to the top of the 52-bit field."""
    out = []
    for b in bits32:
        s, e, m = b >> 31, (b >> 23) & 0xFF, b & 0x7FFFFF
        if e == 0xFF:
            e64 = 0x7FF
        elif e == 0:
            e64 = 0 if m == 0 else 0x001  # keep subnormals below normals, order preserved
        else:
            e64 = e - 127 + 1023
        out.append((s << 63) | (e64 << 52) | (m << 29))
    return out


@pytest.mark.parametrize("width", [16, 32, 64])
def test_float_total_order_of_special_values(width):
    seq = {16: TOTAL_ORDER_F16, 32: TOTAL_ORDER_F32, 64: _widen_f32_to_f64(TOTAL_ORDER_F32)}[width]
    dt = {16: np.uint16, 32: np.uint32, 64: np.uint64}[width]
    want = np.array(seq, dtype=dt)
    rng = np.random.default_rng(width)
    for _ in range(20):
        shuffled = want[rng.permutation(want.size)]
        assert np.array_equal(oracle.sort_ordered(shuffled, key_type="float"), want)
        assert np.array_equal(oracle.sort_ordered(shuffled, key_type="float", descending=True), want[::-1])


@pytest.mark.parametrize("width", [8, 16, 32, 64])
def test_signed_matches_python_sorted(width):
    dt = {8: np.uint8, 16: np.uint16, 32: np.uint32, 64: np.uint64}[width]
    sdt = {8: np.int8, 16: np.int16, 32: np.int32, 64: np.int64}[width]
    rng = np.random.default_rng(100 + width)
    for n in (0, 1, 7, 500):
        k = rng.integers(0, 1 << 63, size=n, dtype=np.uint64).astype(dt)
        k[: n // 3] = k[n // 3: 2 * (n // 3)]  # repeated keys exercise stability
        signed = [int(x) for x in k.view(sdt)]
        for desc in (False, True):
            order = sorted(range(n), key=lambda i: signed[i], reverse=desc)
            ko, vo = oracle.sort_ordered(k, np.arange(n, dtype=np.uint32), key_type="signed", descending=desc)
            assert vo.tolist() == order
            assert np.array_equal(ko, k[order])


@pytest.mark.parametrize("width", [32, 64])
def test_finite_floats_match_numpy_and_python(width):
    fdt = {32: np.float32, 64: np.float64}[width]
    dt = {32: np.uint32, 64: np.uint64}[width]
    rng = np.random.default_rng(7 + width)
    f = (rng.standard_normal(3000) * 10.0 ** rng.integers(-30, 30, 3000)).astype(fdt)
    f[::7] = f[1::7][: f[::7].size]  # repeats
    f[f == 0] = 1.0                  # no zeros: -0 and +0 compare equal as values
    k = f.view(dt)
    assert np.array_equal(oracle.sort_ordered(k, key_type="float").view(fdt), np.sort(f))
    vals = [float(x) for x in f]
    for desc in (False, True):
        order = sorted(range(f.size), key=lambda i: vals[i], reverse=desc)
        _, vo = oracle.sort_ordered(k, np.arange(f.size, dtype=np.uint32), key_type="float", descending=desc)
        assert vo.tolist() == order


@pytest.mark.parametrize("width", [8, 16, 32, 64])
def test_unsigned_matches_counting_sort(width):
    dt = {8: np.uint8, 16: np.uint16, 32: np.uint32, 64: np.uint64}[width]
    rng = np.random.default_rng(200 + width)
    k = rng.integers(0, 1 << 63, size=5000, dtype=np.uint64).astype(dt)
    k[:1000] = k[1000:2000]
    v = np.arange(k.size, dtype=np.uint32)
    ko, vo = oracle.sort_ordered(k, v)
    ek, ev = oracle.sort(k, v)
    assert np.array_equal(ko, ek) and np.array_equal(vo, ev)
    kd, vd = oracle.sort_ordered(k, v, descending=True)
    assert vd.tolist() == sorted(range(k.size), key=lambda i: int(k[i]), reverse=True)


def _zeros_equal(keys, key_type):
    cols = _REAL_COLUMNS(keys, key_type)
    if key_type == "float":
        cols[1] = np.zeros_like(cols[1])  # -0 and +0 tie
    return cols


def _nan_payload_not_reversed(keys, key_type):
    cols = _REAL_COLUMNS(keys, key_type)
    if key_type == "float":
        cols[0] = np.abs(cols[0])  # negative NaNs by ascending payload
    return cols


def _signed_as_unsigned(keys, key_type):
    return _REAL_COLUMNS(keys, "unsigned" if key_type == "signed" else key_type)


_REAL_COLUMNS = oracle._order_columns


def test_signed_8bit_hand_ordered():
    """Every int8 value in two's-complement order, from shuffles, in both
    directions (an 8-bit key has no IEEE format; FLOAT is refused)."""
    want = np.array(list(range(0x80, 0x100)) + list(range(0, 0x80)), dtype=np.uint8)
    rng = np.random.default_rng(8)
    for _ in range(10):
        sh = want[rng.permutation(want.size)]
        assert np.array_equal(oracle.sort_ordered(sh, key_type="signed"), want)
        assert np.array_equal(oracle.sort_ordered(sh, key_type="signed", descending=True), want[::-1])


def _pins_pass():
    try:
        test_signed_8bit_hand_ordered()
        for w in (16, 32, 64):
            test_float_total_order_of_special_values(w)
            test_signed_matches_python_sorted(w)
    except AssertionError:
        return False
    return True


@pytest.mark.parametrize("plant", [_zeros_equal, _nan_payload_not_reversed, _signed_as_unsigned])
def test_planted_mistake_is_caught(monkeypatch, plant):
    """A plausible slip planted in the oracle's order makes a pin fail."""
    assert _pins_pass()
    monkeypatch.setattr(oracle, "_order_columns", plant)
    assert not _pins_pass()


# ---- keys of several 64-bit words -------------------------------------------------

def test_wide_single_word_matches_ordered_sort():
    rng = np.random.default_rng(41)
    k = rng.integers(0, 1 << 63, size=3000, dtype=np.uint64) * np.uint64(2) + rng.integers(0, 2, 3000).astype(np.uint64)
    k[:500] = k[500:1000]
    v = np.arange(k.size, dtype=np.uint32)
    for key_type in ("unsigned", "signed", "float"):
        for desc in (False, True):
            wk, wv = oracle.sort_wide(k.reshape(-1, 1), v, key_type=key_type, descending=desc)
            ek, ev = oracle.sort_ordered(k, v, key_type=key_type, descending=desc)
            assert np.array_equal(wk.ravel(), ek) and np.array_equal(wv, ev), (key_type, desc)


def test_wide_hand_ordered_two_word_keys():
    top, allw = 1 << 63, (1 << 64) - 1
    # (lo, hi) rows in unsigned order of the 128-bit value
    rows = [(0, 0), (5, 0), (allw, 0), (0, 1), (3, 1), (0, top - 1), (0, top), (allw, allw)]
    want = np.array(rows, dtype=np.uint64)
    rng = np.random.default_rng(2)
    shuffled = want[rng.permutation(len(rows))]
    assert np.array_equal(oracle.sort_wide(shuffled), want)
    # two's complement: keys with the top bit set are negative, most negative first
    signed = [want[6], want[7], *want[:6]]
    assert np.array_equal(oracle.sort_wide(shuffled, key_type="signed"), np.array(signed))
    # binary128: -NaN, -inf, -1, -0, +0, 1, +inf, +NaN (hi word holds sign, exponent, top fraction)
    f128 = [(1, 0xFFFF800000000000), (0, 0xFFFF000000000000), (0, 0xBFFF000000000000),
            (0, 0x8000000000000000), (0, 0), (0, 0x3FFF000000000000), (0, 0x7FFF000000000000),
            (1, 0x7FFF800000000000)]
    f = np.array(f128, dtype=np.uint64)
    for _ in range(5):
        sh = f[rng.permutation(len(f128))]
        assert np.array_equal(oracle.sort_wide(sh, key_type="float"), f)
        assert np.array_equal(oracle.sort_wide(sh, key_type="float", descending=True), f[::-1])


# ---- property-based pins (hypothesis) -----------------------------------------------
import struct

from hypothesis import given, settings, strategies as st


@settings(max_examples=200, deadline=None)
@given(st.lists(st.floats(allow_nan=False, width=32), max_size=40), st.booleans())
def test_float32_order_is_python_float_order(values, desc):
    """Non-NaN binary32 values: the oracle's order is Python's float order
    (ties between -0.0 and +0.0 broken by sign, equal bits by position)."""
    bits = np.array([struct.unpack("<I", struct.pack("<f", v))[0] for v in values], dtype=np.uint32)
    key = lambda i: (values[i], 0 if struct.pack("<f", values[i])[3] & 0x80 else 1)  # noqa: E731
    want = sorted(range(len(values)), key=key, reverse=desc)
    _, got = oracle.sort_ordered(bits, np.arange(len(values), dtype=np.uint32), key_type="float", descending=desc)
    assert got.tolist() == want


@settings(max_examples=200, deadline=None)
@given(st.lists(st.integers(min_value=-(1 << 127), max_value=(1 << 127) - 1), max_size=30), st.booleans())
def test_two_word_signed_order_is_python_int_order(values, desc):
    """128-bit two's-complement keys as two little-endian words sort like
    the Python integers they encode."""
    words = np.array([[(v % (1 << 128)) & ((1 << 64) - 1), (v % (1 << 128)) >> 64] for v in values],
                     dtype=np.uint64).reshape(-1, 2)
    want = sorted(range(len(values)), key=lambda i: values[i], reverse=desc)
    _, got = oracle.sort_wide(words, np.arange(len(values), dtype=np.uint32), key_type="signed", descending=desc)
    assert got.tolist() == want
