"""GPU parity of batch stream sorting of 16-bit keys (fs_hist16_accumulate,
fs_hist16_prefix, fs_expand16, fs_sort16_host) against the oracle, byte for
byte.

A stream of batches is sorted exactly when the accumulated histogram equals
the oracle's histogram of the concatenated batches, its prefix equals the
oracle's exclusive scan, and every expanded range equals the same slice of
the oracle's sort of the concatenation.  Batches are ragged, start at
unaligned addresses, include empty and all-equal ones (the packed counters'
wrap repair), and the host driver is run with batch sizes that leave a
ragged last batch, with pinned and pageable memory and in place.
"""
import numpy as np
import pytest
import torch

import fsgen
import oracle
import paper_2605_10390_amd as fs

pytestmark = pytest.mark.gpu


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    return t.cpu().numpy()


def _batches(seed):
    """Ragged batches of every 16-bit distribution, plus an empty one and a
    long all-equal one (more than 2^16 equal keys in one workgroup)."""
    out = []
    sizes = [1, 7, 4096 + 3, 65536 + 5, (1 << 20) + 11, 0, 300_001]
    for i, n in enumerate(sizes):
        dist = fsgen.DISTS_16[i % len(fsgen.DISTS_16)]
        out.append(fsgen.keys_host(dist, 16, n, seed + i))
    out.append(np.full(3 * 65536 + 9, 0xBEEF, dtype=np.uint16))
    return out


def test_accumulated_histogram_prefix_and_expansion(gpu):
    ws = fs.Workspace(gpu)
    batches = _batches(fsgen.seed_for(5, 0))
    hist = fs.new_hist16(gpu)
    for i, b in enumerate(batches):
        # every other batch starts one key past a 16-byte boundary
        t = dev(np.concatenate([np.zeros(1, np.uint16), b]))[1:] if i % 2 else dev(b)
        fs.hist16_accumulate(t, hist, workspace=ws)
    torch.cuda.synchronize()
    assert ws.error_word() == 0
    allk = np.concatenate(batches)
    want_h = oracle.histogram(allk, 0, 16)
    assert np.array_equal(host(hist).view(np.uint64), want_h)

    prefix = fs.hist16_prefix(hist)
    want_p = oracle.exclusive_scan(want_h)
    assert np.array_equal(host(prefix).view(np.uint64), want_p)

    want = oracle.sort(allk)
    n = allk.size
    assert np.array_equal(host(fs.expand16(prefix, 0, n)), want)
    # pieces in any order, unaligned starts and lengths
    rng = np.random.default_rng(3)
    cuts = np.sort(rng.choice(np.arange(1, n), size=40, replace=False))
    bounds = [0, *cuts.tolist(), n]
    pieces = list(zip(bounds[:-1], bounds[1:]))
    rng.shuffle(pieces)
    for a, b in pieces:
        assert np.array_equal(host(fs.expand16(prefix, a, b - a)), want[a:b]), (a, b)


def test_expansion_past_the_total_writes_nothing_there(gpu):
    k = fsgen.keys_host("uniform", 16, 10_000, 17)
    hist = fs.hist16_accumulate(dev(k), fs.new_hist16(gpu))
    prefix = fs.hist16_prefix(hist)
    out = dev(np.full(5000, 0x5A5A, np.uint16))
    fs.expand16(prefix, 8000, 5000, out=out)
    got = host(out)
    assert np.array_equal(got[:2000], oracle.sort(k)[8000:])
    assert np.all(got[2000:] == 0x5A5A)
    # a range that starts past the total writes nothing
    fs.expand16(prefix, 20_000, 100, out=out)
    assert np.array_equal(host(out), got)


def test_empty_histogram_expands_to_nothing(gpu):
    hist = fs.new_hist16(gpu)
    fs.hist16_accumulate(dev(np.zeros(0, np.uint16)), hist)
    prefix = fs.hist16_prefix(hist)
    assert int(prefix[-1].item()) == 0
    out = dev(np.full(64, 7, np.uint16))
    fs.expand16(prefix, 0, 64, out=out)
    assert np.all(host(out) == 7)


@pytest.mark.parametrize("pinned", [True, False])
def test_host_stream_sort_matches_oracle(gpu, pinned):
    ws = fs.Workspace(gpu)
    for di, dist in enumerate(fsgen.DISTS_16):
        n = 3 * (1 << 20) + 12_345
        k = fsgen.keys_host(dist, 16, n, fsgen.seed_for(6, di))
        src = torch.from_numpy(k)
        if pinned:
            src = src.pin_memory()
        # batches of 2^20 + 3 keys (rounded up to a multiple of 8): ragged last batch
        out = fs.sort16_host(src, batch_keys=(1 << 20) + 3, workspace=ws, device=gpu)
        assert np.array_equal(out.numpy(), oracle.sort(k)), (dist, pinned)
        # fewer keys than one batch
        small = fs.sort16_host(src[:1000].clone(), batch_keys=1 << 16, workspace=ws, device=gpu)
        assert np.array_equal(small.numpy(), oracle.sort(k[:1000]))


def test_host_stream_sort_in_place_and_edges(gpu):
    k = fsgen.keys_host("zipf", 16, 2_000_003, 29)
    buf = torch.from_numpy(k.copy()).pin_memory()
    fs.sort16_host(buf, out=buf, batch_keys=1 << 19, device=gpu)
    assert np.array_equal(buf.numpy(), oracle.sort(k))
    empty = torch.from_numpy(np.zeros(0, np.uint16))
    assert fs.sort16_host(empty, device=gpu).numel() == 0
    one = fs.sort16_host(torch.from_numpy(np.array([9], np.uint16)), batch_keys=1, device=gpu)
    assert one.numpy().tolist() == [9]


def test_host_stream_sort_large_is_sorted_permutation(gpu):
    """2^30 host-resident keys (2 GiB) in 2^26-key batches: checked by
    properties that fix the result at any size (non-decreasing, and the
    same multiset as the input, counted on the CPU with numpy).  The keys
    are drawn by the seeded device generator and copied to pinned memory."""
    n = 1 << 30
    src = torch.empty(n, dtype=torch.uint16, pin_memory=True)
    src.copy_(fsgen.keys_device("uniform", 16, n, fsgen.seed_for(1, 0), device=gpu))
    k = src.numpy().copy()
    out = fs.sort16_host(src, batch_keys=1 << 26, device=gpu).numpy()
    step = 1 << 26
    counts_in = np.zeros(65536, np.int64)
    counts_out = np.zeros(65536, np.int64)
    for a in range(0, n, step):
        o = out[a:a + step]
        assert np.all(o[1:] >= o[:-1]), a
        if a:
            assert out[a - 1] <= o[0], a
        counts_in += np.bincount(k[a:a + step], minlength=65536)
        counts_out += np.bincount(o, minlength=65536)
    assert np.array_equal(counts_in, counts_out)


# ---- out-of-core sort of 32- and 64-bit keys (MSD spill) ----------------------------

@pytest.mark.parametrize("bits", [32, 64])
def test_host_sort_wide_keys_matches_oracle(gpu, bits):
    """Several device ranges (device_keys far below n), ragged batches, the
    three wide distributions (uniform; values below 2^20, whose top bits all
    agree; 90% from 256 hot values), against the oracle byte for byte."""
    ws = fs.Workspace(gpu)
    for di, dist in enumerate(fsgen.DISTS_WIDE):
        n = 3 * (1 << 20) + 4321
        k = fsgen.keys_host(dist, bits, n, fsgen.seed_for(7, di))
        src = torch.from_numpy(k).pin_memory()
        out = fs.sort_host(src, batch_keys=(1 << 20) + 3, device_keys=1 << 19, workspace=ws, device=gpu)
        assert np.array_equal(out.numpy(), oracle.sort(k)), (bits, dist)
        assert ws.error_word() == 0


def test_host_sort_wide_edges(gpu):
    rng = np.random.default_rng(4)
    for bits, dt in ((32, np.uint32), (64, np.uint64)):
        for n in (0, 1, 7, 1000):
            k = rng.integers(0, 1 << 63, n, dtype=np.uint64).astype(dt)
            out = fs.sort_host(torch.from_numpy(k), batch_keys=64, device_keys=256, device=gpu)
            assert np.array_equal(out.numpy(), np.sort(k)), (bits, n)
        eq = np.full(100_000, 0xDEADBEEF, dtype=dt)  # every key equal: a copy
        assert np.array_equal(fs.sort_host(torch.from_numpy(eq), device_keys=16, device=gpu).numpy(), eq)


def test_host_sort_splits_oversized_bins(gpu):
    """Window bins holding more keys than one device range are split again
    by their next 16 bits, down to single key values (written out as runs)."""
    rng = np.random.default_rng(8)
    # skewed 32-bit keys: hot values share window bins past the range size
    k = fsgen.keys_host("hot90", 32, 200_000, 3)
    out = fs.sort_host(torch.from_numpy(k), batch_keys=1 << 16, device_keys=1024, device=gpu)
    assert np.array_equal(out.numpy(), oracle.sort(k))
    # one 64-bit value holds 60% of the keys: every level's bin of it is too
    # big, down to the lowest 16 bits, where it is one value
    n = 200_003
    k = rng.integers(0, 1 << 63, n, dtype=np.uint64) * np.uint64(2) + rng.integers(0, 2, n, dtype=np.uint64)
    k[rng.random(n) < 0.6] = np.uint64(0x0123456789ABCDEF)
    out = fs.sort_host(torch.from_numpy(k), batch_keys=1 << 15, device_keys=4096, device=gpu)
    assert np.array_equal(out.numpy(), oracle.sort(k))
    # half the keys share their top 32 bits and differ below: split twice,
    # then ranges that fit
    k = rng.integers(0, 1 << 63, n, dtype=np.uint64)
    half = rng.random(n) < 0.5
    k[half] = (np.uint64(0xCAFEF00D) << np.uint64(32)) | rng.integers(0, 1 << 32, int(half.sum()), dtype=np.uint64)
    out = fs.sort_host(torch.from_numpy(k), batch_keys=1 << 15, device_keys=4096, device=gpu)
    assert np.array_equal(out.numpy(), oracle.sort(k))


@pytest.mark.parametrize("key_type,desc", [("signed", False), ("unsigned", True)])
def test_host_sort_split_bins_in_other_orders(gpu, key_type, desc):
    rng = np.random.default_rng(21)
    n = 100_001
    k = rng.integers(0, 1 << 32, n, dtype=np.uint64).astype(np.uint32)
    k[rng.random(n) < 0.5] = np.uint32(0x80000001)  # one value past the range size, sign bit set
    out = fs.sort_host(torch.from_numpy(k), batch_keys=1 << 14, device_keys=2048, key_type=key_type,
                       descending=desc, device=gpu)
    assert np.array_equal(out.numpy(), oracle.sort_ordered(k, key_type=key_type, descending=desc))


def test_host_sort_wide_large_matches_threaded_oracle(gpu):
    """2^30 host-resident u32 keys (4 GiB) through 2^28-key device ranges,
    against the oracle (its threaded variant, pinned byte-equal to the
    single-threaded one)."""
    n = 1 << 30
    src = torch.empty(n, dtype=torch.uint32, pin_memory=True)
    src.copy_(fsgen.keys_device("uniform", 32, n, fsgen.seed_for(7, 9), device=gpu))
    out = fs.sort_host(src, batch_keys=1 << 26, device_keys=1 << 28, device=gpu)
    want = oracle.sort_mt(src.numpy(), threads=16)
    assert np.array_equal(out.numpy(), want)


# ---- key orders in the stream and out-of-core sorts ------------------------------

ORDERS = [("signed", False), ("float", False), ("float", True), ("unsigned", True)]


@pytest.mark.parametrize("key_type,desc", ORDERS)
def test_stream_sorts_in_every_order(gpu, key_type, desc):
    """The accumulated histogram / expansion, the 16-bit host sort and the
    out-of-core 32/64-bit sort, each in another key order, against
    oracle.sort_ordered (random bit patterns: floats include NaNs,
    infinities and both zeros)."""
    rng = np.random.default_rng(31)
    n = (1 << 20) + 333
    k16 = rng.integers(0, 1 << 16, n, dtype=np.uint64).astype(np.uint16)
    want16 = oracle.sort_ordered(k16, key_type=key_type, descending=desc)
    hist = fs.new_hist16(gpu)
    for a in range(0, n, 300_000):
        fs.hist16_accumulate(dev(k16[a:a + 300_000]), hist, key_type=key_type, descending=desc)
    prefix = fs.hist16_prefix(hist)
    assert np.array_equal(host(fs.expand16(prefix, 0, n, key_type=key_type, descending=desc)), want16)
    part = host(fs.expand16(prefix, 1000, 5000, key_type=key_type, descending=desc))
    assert np.array_equal(part, want16[1000:6000])
    out16 = fs.sort16_host(torch.from_numpy(k16).pin_memory(), batch_keys=1 << 18, device=gpu,
                           key_type=key_type, descending=desc)
    assert np.array_equal(out16.numpy(), want16)
    for bits, dt in ((32, np.uint32), (64, np.uint64)):
        k = rng.integers(0, 1 << 63, n, dtype=np.uint64).astype(dt) * dt(2) + rng.integers(0, 2, n).astype(dt)
        out = fs.sort_host(torch.from_numpy(k).pin_memory(), batch_keys=1 << 18, device_keys=1 << 18,
                           device=gpu, key_type=key_type, descending=desc)
        assert np.array_equal(out.numpy(), oracle.sort_ordered(k, key_type=key_type, descending=desc)), bits
