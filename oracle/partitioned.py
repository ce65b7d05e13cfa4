"""Partitioned oracle for inputs larger than one sort the host can hold at once.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The sorted output of n keys is cut, in key order, into value ranges of at
most `cap` keys each.  A range's part of the output is the sort of the keys
that fall in it, and it starts at the number of keys below the range.  So
the whole sorted array is checked range by range: collect a range's keys in
input order, sort them with the oracle's counting sort (`oracle.sort`, the
radix phases of Sec. II), and compare with the output at that offset.  The
ranges come from the oracle's own 16-bit digit histograms (Sec. III-B.1,
Alg. 1): the top 16 bits first; a bin holding more than `cap` keys is split
again by its next 16 bits (as for 64-bit keys below 2^20, where every key
shares its top 44 bits), down to single key values, whose range is then a
run of equal keys checked without sorting.  Every step is a plain count or
a plain counting sort, so the result is exact.
"""
from concurrent.futures import ThreadPoolExecutor

import numpy as np

from . import histogram, sort

DIGIT = 16
BINS = 1 << DIGIT


def _chunks(keys, chunk):
    for a in range(0, keys.size, chunk):
        yield a, keys[a:a + chunk]


def _window_hist(keys, key_bits, prefix, shift, chunk, pool):
    """Histogram of bits [shift-16, shift) over the keys whose bits from
    `shift` up equal `prefix` (all keys when shift == key_bits)."""
    def one(piece):
        if shift < key_bits:
            piece = piece[(piece.astype(np.uint64, copy=False) >> np.uint64(shift)) == np.uint64(prefix)]
        return histogram(piece, shift - DIGIT, DIGIT)
    total = np.zeros(BINS, dtype=np.uint64)
    for h in pool.map(one, [c for _, c in _chunks(keys, chunk)]):
        total += h
    return total


class Plan:
    """Value ranges in key order.  ranges[i] = (count, single_value or None);
    a lookup from key to range id goes through 16-bit tables: table 0 reads
    the top window; an entry >= 0 is a range id, -1 - j sends the key to
    table j (a split bin), which reads the next 16 bits."""

    def __init__(self):
        self.ranges = []
        self.tables = []  # (shift of the window's low bit, int64[BINS])

    def range_ids(self, keys):
        k = keys.astype(np.uint64, copy=False)
        shift, table = self.tables[0]
        ids = table[((k >> np.uint64(shift)) & np.uint64(BINS - 1)).astype(np.int64)]
        while True:
            todo = np.nonzero(ids < 0)[0]
            if not todo.size:
                return ids
            sub = -1 - ids[todo]
            for j in np.nonzero(np.bincount(sub, minlength=len(self.tables)))[0]:
                sel = todo if sub.size and sub[0] == j and np.all(sub == j) else todo[sub == j]
                shift, table = self.tables[int(j)]
                ids[sel] = table[((k[sel] >> np.uint64(shift)) & np.uint64(BINS - 1)).astype(np.int64)]


def plan_ranges(keys, key_bits, cap, chunk=1 << 26, threads=8):
    """Cut the key space of `keys` into ranges of at most `cap` keys (a
    single key value may exceed it), in key order."""
    plan = Plan()
    with ThreadPoolExecutor(threads) as pool:
        def visit(prefix, shift):
            h = _window_hist(keys, key_bits, prefix, shift, chunk, pool)
            low = shift - DIGIT
            table = np.empty(BINS, dtype=np.int64)
            t_index = len(plan.tables)
            plan.tables.append((low, table))
            cur = -1  # open range id
            for b in range(BINS):
                c = int(h[b])
                if c > cap:
                    cur = -1
                    if low > 0:
                        table[b] = -1 - len(plan.tables)
                        visit((prefix << DIGIT) | b, low)
                    else:
                        table[b] = len(plan.ranges)
                        plan.ranges.append([c, (prefix << DIGIT) | b])
                    continue
                if cur < 0 or plan.ranges[cur][0] + c > cap:
                    cur = len(plan.ranges)
                    plan.ranges.append([0, None])
                plan.ranges[cur][0] += c
                table[b] = cur
            plan.tables[t_index] = (low, table)
        visit(0, key_bits)
    return plan


def partitioned_sort(keys, key_bits, cap, chunk=1 << 26, threads=8):
    """Yield (offset, expected) for every range of plan_ranges(keys, ...),
    in key order: `expected` is the oracle's sort of the range's keys, to be
    found at sorted positions [offset, offset + len(expected)).  A range of
    one key value over `cap` keys yields a lazy constant instead
    (np.broadcast_to), so its keys are never copied."""
    keys = np.ascontiguousarray(keys)
    plan = plan_ranges(keys, key_bits, cap, chunk, threads)
    R = len(plan.ranges)
    gather = [r[1] is None for r in plan.ranges]
    pieces = [[] for _ in range(R)]

    def split(piece):
        ids = plan.range_ids(piece)
        if R <= BINS:
            # group by range id with the oracle's stable counting sort: the
            # 16-bit id is the key and the key rides as the payload, so
            # input order is kept inside every range
            ids_sorted, grouped = sort(ids.astype(np.uint16), piece.astype(np.uint64, copy=False))
            grouped = grouped.astype(piece.dtype, copy=False)
            bounds = np.searchsorted(ids_sorted, np.arange(R + 1), side="left")
        else:
            order = np.argsort(ids, kind="stable")
            grouped = piece[order]
            bounds = np.searchsorted(ids[order], np.arange(R + 1), side="left")
        return [(r, grouped[bounds[r]:bounds[r + 1]]) for r in range(R)
                if bounds[r + 1] > bounds[r] and gather[r]]

    with ThreadPoolExecutor(threads) as pool:
        for parts in pool.map(split, [c for _, c in _chunks(keys, chunk)]):
            for r, p in parts:
                pieces[r].append(p)

        def one(r):
            if not gather[r]:
                return np.broadcast_to(np.array(plan.ranges[r][1], dtype=keys.dtype), (plan.ranges[r][0],))
            got = np.concatenate(pieces[r]) if pieces[r] else np.empty(0, dtype=keys.dtype)
            pieces[r] = None
            assert got.size == plan.ranges[r][0]
            return sort(got)

        offset = 0
        for r0 in range(0, R, threads):
            for r, expected in zip(range(r0, min(R, r0 + threads)),
                                   pool.map(one, range(r0, min(R, r0 + threads)))):
                yield offset, expected
                offset += plan.ranges[r][0]
