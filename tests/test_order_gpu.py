"""GPU parity of the key orders (FS_FLAG_SIGNED, FS_FLAG_FLOAT,
FS_FLAG_DESCENDING) against oracle.sort_ordered, byte for byte.

Every width takes both of its paths (16-bit keys-only: compressed histogram
and expansion; 16-bit pairs: histogram, payload passes, expansion; wider
keys: the 8-bit digit passes), over random bit patterns (for floats these
include NaNs, infinities, subnormals and both zeros) with IEEE special
values and repeated keys mixed in, sizes spanning several tiles with ragged
tails, and all-equal keys (every digit trivial: a copy)."""
import numpy as np
import pytest
import torch

import fsgen
import oracle
import paper_2605_10390_amd as fs
from tests.test_oracle_order_pins import TOTAL_ORDER_F16, TOTAL_ORDER_F32, _widen_f32_to_f64

pytestmark = pytest.mark.gpu

SIZES = [1, 63, 4097, 3 * 4096 + 17, 65536 + 123, (1 << 20) + 7]
ORDERS = [("signed", False), ("signed", True), ("float", False), ("float", True), ("unsigned", True)]
SPECIALS = {16: TOTAL_ORDER_F16, 32: TOTAL_ORDER_F32, 64: _widen_f32_to_f64(TOTAL_ORDER_F32)}


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    return t.cpu().numpy()


def _keys(bits, n, seed):
    k = fsgen.keys_host("uniform", bits, n, seed)
    if n >= 64:
        sp = np.array(SPECIALS[bits], dtype=k.dtype)
        rng = np.random.default_rng(seed)
        pos = rng.choice(n, size=min(n // 4, 4 * sp.size), replace=False)
        k[pos] = sp[np.arange(pos.size) % sp.size]
        k[: n // 8] = k[n // 8: 2 * (n // 8)]  # repeats: stability
    return k


@pytest.mark.parametrize("bits", [16, 32, 64])
@pytest.mark.parametrize("key_type,desc", ORDERS)
def test_keys_in_every_order(gpu, bits, key_type, desc):
    ws = fs.Workspace(gpu)
    for n in SIZES:
        k = _keys(bits, n, fsgen.seed_for(7, bits) + n)
        out = fs.sort_keys(dev(k), workspace=ws, key_type=key_type, descending=desc)
        torch.cuda.synchronize()
        assert ws.error_word() == 0
        assert np.array_equal(host(out), oracle.sort_ordered(k, key_type=key_type, descending=desc)), n


@pytest.mark.parametrize("bits", [16, 32, 64])
@pytest.mark.parametrize("key_type,desc", ORDERS)
def test_pairs_in_every_order(gpu, bits, key_type, desc):
    ws = fs.Workspace(gpu)
    for n in SIZES:
        k = _keys(bits, n, fsgen.seed_for(8, bits) + n)
        v = fsgen.vals_host(n, 4)
        ko, vo = fs.sort_pairs(dev(k), dev(v), workspace=ws, key_type=key_type, descending=desc)
        ek, ev = oracle.sort_ordered(k, v, key_type=key_type, descending=desc)
        assert ws.error_word() == 0
        assert np.array_equal(host(ko), ek), n
        assert np.array_equal(host(vo), ev), n


def test_dtype_picks_the_order(gpu):
    rng = np.random.default_rng(5)
    f = rng.standard_normal(10_000).astype(np.float32)
    out = fs.sort_keys(dev(f))
    assert np.array_equal(host(out), np.sort(f))
    i = rng.integers(-(1 << 40), 1 << 40, 10_000, dtype=np.int64)
    assert np.array_equal(host(fs.sort_keys(dev(i), descending=True)), np.sort(i)[::-1])
    h = rng.standard_normal(5000).astype(np.float16)
    h[h == 0] = 1
    assert np.array_equal(host(fs.sort_keys(dev(h))), np.sort(h))


@pytest.mark.parametrize("bits", [16, 32, 64])
def test_all_equal_keys_any_order(gpu, bits):
    k = np.full(70_001, SPECIALS[bits][3], dtype=fsgen.key_dtype(bits))
    v = fsgen.vals_host(k.size, 4)
    for key_type, desc in ORDERS:
        ko, vo = fs.sort_pairs(dev(k), dev(v), key_type=key_type, descending=desc)
        assert np.array_equal(host(ko), k) and np.array_equal(host(vo), v)


# (key bits, payload bytes, n): every bin of the segmented sort at the
# default tuning -- the LDS bin, the 16-bit-digit bin (one workgroup, and
# split into parts from 2^18 keys), the one-workgroup bin and the large bin
SEGMENTS = [(16, 0, 100), (16, 0, 20_000), (16, 0, 300_001), (16, 4, 5_000), (16, 4, 200_003),
            (32, 0, 3_000), (32, 0, 50_001), (32, 0, 400_007), (64, 4, 2_000), (64, 4, 100_003),
            (64, 0, 300_001), (32, 8, 1), (64, 0, 0)]


@pytest.mark.parametrize("key_type,desc", ORDERS)
def test_segmented_in_every_order(gpu, key_type, desc):
    rng = np.random.default_rng(11)
    segs, want = [], []
    for i, (bits, vb, n) in enumerate(SEGMENTS):
        k = _keys(bits, n, fsgen.seed_for(9, i) + n)
        v = rng.integers(0, 1 << 32, n, dtype=np.uint64).astype(np.uint32 if vb == 4 else np.uint64) if vb else None
        ki = dev(k)
        vi = dev(v) if vb else None
        segs.append((ki, torch.empty_like(ki), vi, torch.empty_like(vi) if vb else None))
        want.append(oracle.sort_ordered(k, v, key_type=key_type, descending=desc))
    ws = fs.sort_segmented(segs, key_type=key_type, descending=desc)
    torch.cuda.synchronize()
    assert ws.error_word() == 0
    for i, ((_, ko, _, vo), w) in enumerate(zip(segs, want)):
        if vo is None:
            assert np.array_equal(host(ko), w), SEGMENTS[i]
        else:
            assert np.array_equal(host(ko), w[0]), SEGMENTS[i]
            assert np.array_equal(host(vo), w[1]), SEGMENTS[i]


@pytest.mark.parametrize("words", [1, 2, 3])
@pytest.mark.parametrize("key_type", ["unsigned", "signed", "float"])
def test_wide_keys_match_oracle(gpu, words, key_type):
    """Keys of several 64-bit words, against the oracle's whole-width
    integer comparison; repeated keys and keys equal in their low words
    check stability and the word order."""
    rng = np.random.default_rng(17 * words)
    ws = fs.Workspace(gpu)
    for n in (1, 1000, 70_001):
        k = rng.integers(0, 1 << 63, size=(n, words), dtype=np.uint64) * np.uint64(2)
        k += rng.integers(0, 2, size=(n, words)).astype(np.uint64)
        if n > 10:
            k[: n // 4] = k[n // 4: n // 2]          # whole-key repeats
            k[n // 2: n // 2 + n // 8, 1:] = k[0, 1:]  # equal high words, differing low words
            k[-n // 8:, :-1] = 7                      # equal low words, differing high words
        v = rng.integers(0, 1 << 32, n, dtype=np.uint64).astype(np.uint32)
        for desc in (False, True):
            got = fs.sort_wide(dev(k), workspace=ws, key_type=key_type, descending=desc)
            assert np.array_equal(host(got), oracle.sort_wide(k, key_type=key_type, descending=desc)), (n, desc)
            gk, gv = fs.sort_wide(dev(k), dev(v), workspace=ws, key_type=key_type, descending=desc)
            ek, ev = oracle.sort_wide(k, v, key_type=key_type, descending=desc)
            assert ws.error_word() == 0
            assert np.array_equal(host(gk), ek) and np.array_equal(host(gv), ev), (n, desc)


@pytest.mark.parametrize("key_type,desc", [("unsigned", False), ("unsigned", True), ("signed", False),
                                           ("signed", True)])
def test_8bit_keys_and_pairs(gpu, key_type, desc):
    """8-bit keys (one digit): keys only and with 4- and 8-byte payloads,
    across tile boundaries with ragged tails, unaligned starts, skewed and
    all-equal keys."""
    rng = np.random.default_rng(8)
    ws = fs.Workspace(gpu)
    for n in (1, 15, 17, 4095, 4097, 3 * 4096 + 5, 65536 + 7, (1 << 20) + 3):
        k = rng.integers(0, 256, n, dtype=np.uint64).astype(np.uint8)
        if n > 100:
            k[: n // 3] = 200  # a hot value
        for off in (0, 3):
            kk = dev(np.concatenate([np.zeros(off, np.uint8), k]))[off:]
            got = fs.sort_keys(kk, workspace=ws, key_type=key_type, descending=desc)
            assert np.array_equal(host(got), oracle.sort_ordered(k, key_type=key_type, descending=desc)), (n, off)
        for vdt in (np.uint32, np.uint64):
            v = rng.integers(0, 1 << 32, n, dtype=np.uint64).astype(vdt)
            gk, gv = fs.sort_pairs(dev(k), dev(v), workspace=ws, key_type=key_type, descending=desc)
            ek, ev = oracle.sort_ordered(k, v, key_type=key_type, descending=desc)
            assert ws.error_word() == 0
            assert np.array_equal(host(gk), ek) and np.array_equal(host(gv), ev), (n, vdt)
    eq = np.full(70_000, 9, np.uint8)
    assert np.array_equal(host(fs.sort_keys(dev(eq), key_type=key_type, descending=desc)), eq)
