"""Invariant checker for sort results, independent of the oracle and of the
HIP path.

For a payload equal to the original index these four properties pin the
unique stable ascending result:
  1. vals_out is a permutation of 0 .. n-1;
  2. keys_out[i] == keys_in[vals_out[i]];
  3. keys_out is non-decreasing;
  4. vals_out strictly increases inside every run of equal keys.
"""
import numpy as np


def check_index_pairs(keys_in, keys_out, vals_out):
    """Raise AssertionError unless (keys_out, vals_out) is the stable sort of
    keys_in with payload 0..n-1."""
    n = keys_in.size
    assert keys_out.size == n and vals_out.size == n, "length changed"
    if n == 0:
        return
    v = vals_out.astype(np.int64)
    assert v.min() >= 0 and v.max() < n, "payload out of range"
    seen = np.zeros(n, dtype=np.uint8)
    seen[v] = 1
    assert seen.all(), "payload is not a permutation"
    assert np.array_equal(keys_in[v], keys_out), "keys do not travel with their payload"
    ko = keys_out
    assert np.all(ko[1:] >= ko[:-1]), "keys not non-decreasing"
    eq = ko[1:] == ko[:-1]
    assert np.all(v[1:][eq] > v[:-1][eq]), "equal keys out of input order"


def check_keys(keys_in, keys_out, key_bits):
    """Raise AssertionError unless keys_out is keys_in in ascending order
    (multiset compared through np.unique counts)."""
    assert keys_out.size == keys_in.size, "length changed"
    if keys_in.size == 0:
        return
    assert np.all(keys_out[1:] >= keys_out[:-1]), "keys not non-decreasing"
    ui, ci = np.unique(keys_in, return_counts=True)
    uo, co = np.unique(keys_out, return_counts=True)
    assert np.array_equal(ui, uo) and np.array_equal(ci, co), "multiset changed"
