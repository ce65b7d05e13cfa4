"""CPU oracle for the sort: plain C counting sort behind ctypes.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
``bench.py``'s ``cpu_baseline`` leg may import this package.  The product
path (``paper_2605_10390_amd``) never imports it.

Each function follows a passage of the paper (arXiv 2605.10390):
  histogram       -- leaf counters of a digit (Sec. III-B.1, Alg. 1)
  exclusive_scan  -- GetIndex as the exclusive prefix (Alg. 3)
  select          -- GetItem as an order-statistic walk (Alg. 2)
  expand          -- the sorted array written out from a full-width
                     histogram (Alg. 5 with no trailing bits)
  sort            -- histogram / prefix / stable scatter radix sort
                     (Sec. II), least-significant 8-bit digit first
  sort_mt         -- `sort` split over threads (contiguous chunks, blocks
                     laid out value-major then thread-minor), for timing
  sort_segments   -- independent sorts of back-to-back segments
  sort_wide       -- stable sort of keys of several 64-bit words, compared
                     as Python integers of the whole width (unsigned,
                     two's complement, or sign-magnitude)
  sort_ordered    -- the same stable sort under another key order: signed
                     integers, IEEE 754 totalOrder of floats, descending
                     (the paper's keys of any precision, Sec. I); written
                     from those orders' definitions, not from a bit mapping
  partitioned.partitioned_sort -- the sort of an input too large for one
                     oracle sort, cut in key order into value ranges from
                     16-bit digit histograms and sorted range by range
Every function is pinned by tests/test_oracle_pins.py against brute force,
closed forms and library routines (the partitioned sort by
tests/test_oracle_partitioned.py); none is "parity unpinned".
"""
import ctypes
import os

import numpy as np

from . import build as _build

_lib = None

_KEY_DTYPES = {1: np.uint8, 2: np.uint16, 4: np.uint32, 8: np.uint64}


def load(path=None, rebuild_if_missing=True):
    """Load liboracle.so (compiling it with gcc when it is missing)."""
    global _lib
    if path is None and _lib is not None:
        return _lib
    p = path or _build.LIB
    if not os.path.exists(p):
        if not rebuild_if_missing:
            raise FileNotFoundError(p)
        _build.build(p)
    lib = ctypes.CDLL(p)
    u64, vp, i32 = ctypes.c_uint64, ctypes.c_void_p, ctypes.c_int
    lib.oracle_histogram.argtypes = [vp, u64, i32, i32, i32, vp]
    lib.oracle_histogram.restype = i32
    lib.oracle_exclusive_scan.argtypes = [vp, u64, vp]
    lib.oracle_exclusive_scan.restype = i32
    lib.oracle_select.argtypes = [vp, u64, u64]
    lib.oracle_select.restype = u64
    lib.oracle_expand.argtypes = [vp, u64, vp, i32]
    lib.oracle_expand.restype = i32
    lib.oracle_sort.argtypes = [vp, vp, vp, vp, u64, i32, i32]
    lib.oracle_sort.restype = i32
    lib.oracle_sort_mt.argtypes = [vp, vp, vp, vp, u64, i32, i32, i32]
    lib.oracle_sort_mt.restype = i32
    lib.oracle_sort_segments.argtypes = [vp, vp, vp, vp, u64, vp, vp, vp, vp, i32]
    lib.oracle_sort_segments.restype = i32
    if path is None:
        _lib = lib
    return lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None and a.size else None


def _check(rc, what):
    if rc != 0:
        raise RuntimeError(f"oracle {what} failed with code {rc}")


def histogram(keys, shift, bits, lib=None):
    """Counts of the `bits`-wide digit at bit `shift`: uint64[2**bits]."""
    lib = lib or load()
    keys = np.ascontiguousarray(keys)
    h = np.zeros(1 << bits, dtype=np.uint64)
    _check(lib.oracle_histogram(_ptr(keys), keys.size, keys.itemsize, shift, bits, _ptr(h)),
           "histogram")
    return h


def exclusive_scan(hist, lib=None):
    """prefix[b] = sum(hist[:b]); the extra last entry is the total."""
    lib = lib or load()
    hist = np.ascontiguousarray(hist, dtype=np.uint64)
    p = np.zeros(hist.size + 1, dtype=np.uint64)
    _check(lib.oracle_exclusive_scan(_ptr(hist), hist.size, p.ctypes.data_as(ctypes.c_void_p)),
           "exclusive_scan")
    return p


def select(hist, index, lib=None):
    """Value at sorted position `index`; len(hist) when out of range."""
    lib = lib or load()
    hist = np.ascontiguousarray(hist, dtype=np.uint64)
    return int(lib.oracle_select(_ptr(hist), hist.size, int(index)))


def expand(hist, key_dtype, lib=None):
    """Sorted array implied by a histogram over every key value."""
    lib = lib or load()
    hist = np.ascontiguousarray(hist, dtype=np.uint64)
    out = np.empty(int(hist.sum()), dtype=key_dtype)
    _check(lib.oracle_expand(_ptr(hist), hist.size, _ptr(out), out.itemsize), "expand")
    return out


def sort(keys, vals=None, lib=None):
    """Stable ascending sort; returns keys_out or (keys_out, vals_out)."""
    lib = lib or load()
    keys = np.ascontiguousarray(keys)
    ko = np.empty_like(keys)
    if vals is None:
        _check(lib.oracle_sort(_ptr(keys), _ptr(ko), None, None, keys.size, keys.itemsize, 0),
               "sort")
        return ko
    vals = np.ascontiguousarray(vals)
    if vals.size != keys.size:
        raise ValueError("keys and vals differ in length")
    vo = np.empty_like(vals)
    _check(lib.oracle_sort(_ptr(keys), _ptr(ko), _ptr(vals), _ptr(vo), keys.size,
                           keys.itemsize, vals.itemsize), "sort")
    return ko, vo


def sort_mt(keys, vals=None, threads=4, lib=None):
    """`sort` split over `threads` threads (for timing the CPU baseline);
    byte-equal to `sort`."""
    lib = lib or load()
    keys = np.ascontiguousarray(keys)
    ko = np.empty_like(keys)
    if vals is None:
        _check(lib.oracle_sort_mt(_ptr(keys), _ptr(ko), None, None, keys.size, keys.itemsize, 0, int(threads)),
               "sort_mt")
        return ko
    vals = np.ascontiguousarray(vals)
    if vals.size != keys.size:
        raise ValueError("keys and vals differ in length")
    vo = np.empty_like(vals)
    _check(lib.oracle_sort_mt(_ptr(keys), _ptr(ko), _ptr(vals), _ptr(vo), keys.size, keys.itemsize,
                              vals.itemsize, int(threads)), "sort_mt")
    return ko, vo


def sort_segments(segments, lib=None):
    """Sort each (keys[, vals]) array of `segments` independently."""
    out = []
    for seg in segments:
        if isinstance(seg, tuple):
            out.append(sort(seg[0], seg[1], lib=lib))
        else:
            out.append(sort(seg, lib=lib))
    return out


_SIGNED = {1: np.int8, 2: np.int16, 4: np.int32, 8: np.int64}
_FLOAT = {2: np.float16, 4: np.float32, 8: np.float64}


def _order_columns(keys, key_type):
    """Sort columns for numpy.lexsort (last = most significant) that rank
    `keys` (unsigned words) in the order of `key_type`."""
    if key_type == "unsigned":
        return [keys]
    if key_type == "signed":
        return [keys.view(_SIGNED[keys.itemsize])]
    if key_type != "float":
        raise ValueError(key_type)
    # IEEE 754 totalOrder: negative NaNs (larger payload first), then the
    # numbers by value with -0 before +0, then positive NaNs (smaller
    # payload first)
    f = keys.view(_FLOAT[keys.itemsize])
    negative = np.signbit(f)
    nan = np.isnan(f)
    cls = np.where(nan, np.where(negative, 0, 2), 1)
    # NaNs are masked before the cast (their order comes from cls and
    # nan_rank), so no NaN is ever converted
    value = np.zeros(f.shape, dtype=np.float64)
    value[~nan] = f[~nan].astype(np.float64)
    zero_sign = np.where((f == 0) & ~negative, 1, 0)
    payload = (keys.astype(np.uint64) & np.uint64((1 << (8 * keys.itemsize - 1)) - 1)).astype(np.int64)
    nan_rank = np.where(nan, np.where(negative, -payload, payload), 0)
    return [nan_rank, zero_sign, value, cls]


def sort_ordered(keys, vals=None, key_type="unsigned", descending=False):
    """Stable sort of unsigned key words read as `key_type` ("unsigned",
    "signed" two's complement, or "float" = IEEE 754 binary16/32/64 in
    totalOrder), ascending or descending; equal keys (equal bits) keep their
    input order either way.  Returns keys_out or (keys_out, vals_out)."""
    keys = np.ascontiguousarray(keys)
    n = keys.size
    if descending:
        # a stable ascending sort of the reversed input, read backwards
        rev = keys[::-1].copy()
        idx = np.lexsort(_order_columns(rev, key_type))
        perm = (n - 1 - idx)[::-1]
    else:
        perm = np.lexsort(_order_columns(keys, key_type))
    if vals is None:
        return keys[perm]
    vals = np.ascontiguousarray(vals)
    if vals.size != n:
        raise ValueError("keys and vals differ in length")
    return keys[perm], vals[perm]


def _wide_value(words, key_type):
    """A key of 64-bit words (least significant first) as a sortable Python
    value of the whole width."""
    bits = 64 * len(words)
    v = 0
    for i, w in enumerate(words):
        v |= int(w) << (64 * i)
    if key_type == "unsigned":
        return v
    if key_type == "signed":
        return v - (1 << bits) if v >> (bits - 1) else v
    if key_type == "float":
        # sign-magnitude total order: negatives by falling magnitude, -0 before +0
        mag = v & ((1 << (bits - 1)) - 1)
        return (0, -mag) if v >> (bits - 1) else (1, mag)
    raise ValueError(key_type)


def sort_wide(keys, vals=None, key_type="unsigned", descending=False):
    """Stable sort of an (n, W) uint64 array of keys (word 0 least
    significant) by the whole-width value of `key_type`; equal keys keep
    their input order in either direction.  Returns keys_out or
    (keys_out, vals_out)."""
    keys = np.ascontiguousarray(keys, dtype=np.uint64)
    vals_of = [_wide_value(row, key_type) for row in keys]
    order = sorted(range(keys.shape[0]), key=lambda i: vals_of[i], reverse=descending)
    if vals is None:
        return keys[order]
    vals = np.ascontiguousarray(vals)
    return keys[order], vals[order]
