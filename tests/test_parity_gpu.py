"""GPU parity: every result of the HIP path equals the CPU oracle's, byte
for byte (integer work: bit-exact, tolerance 0), on the same seeded inputs.

Sizes span several tiles (a scatter tile is 4096 keys) with ragged tails,
every key width and payload width, every distribution of the configs, and
the edge cases: n = 0 and 1, unaligned buffers, all-equal keys (every digit
trivial, the sort is a copy) and a size whose tile offsets span every level
of the offset scan.
"""
import numpy as np
import pytest
import torch

import fsgen
import oracle
import paper_2605_10390_amd as fs
from tests.checks import check_index_pairs

pytestmark = pytest.mark.gpu

SIZES = [1, 2, 63, 64, 65, 4095, 4096, 4097, 3 * 4096 + 17, 65536 + 123, (1 << 20) + 7]


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    return t.cpu().numpy()


def _vals(n, vb, seed):
    return fsgen.vals_host(n, vb, kind="random", seed=seed)


@pytest.mark.parametrize("bits", [16, 32, 64])
def test_keys_match_oracle(gpu, bits):
    ws = fs.Workspace(gpu)
    for n in SIZES:
        for di, dist in enumerate(fsgen.valid_dists(bits)):
            seed = fsgen.seed_for(9, di) + n
            k = fsgen.keys_host(dist, bits, n, seed)
            out = fs.sort_keys(dev(k), workspace=ws)
            torch.cuda.synchronize()
            assert ws.error_word() == 0
            assert np.array_equal(host(out), oracle.sort(k)), (bits, n, dist)


@pytest.mark.parametrize("bits", [16, 32, 64])
@pytest.mark.parametrize("vb", [4, 8])
def test_pairs_match_oracle(gpu, bits, vb):
    ws = fs.Workspace(gpu)
    for n in SIZES:
        for di, dist in enumerate(fsgen.valid_dists(bits)):
            seed = fsgen.seed_for(8, di) + n
            k = fsgen.keys_host(dist, bits, n, seed)
            v = _vals(n, vb, seed)
            ko, vo = fs.sort_pairs(dev(k), dev(v), workspace=ws)
            ek, ev = oracle.sort(k, v)
            assert ws.error_word() == 0
            assert np.array_equal(host(ko), ek), (bits, vb, n, dist)
            assert np.array_equal(host(vo), ev), (bits, vb, n, dist)


def _clobber_keys(bits, dist, n, seed):
    if bits == 8:
        rng = np.random.default_rng(seed)
        if dist == "equal":
            return np.full(n, 0x5A, dtype=np.uint8)
        return rng.integers(0, 256, size=n, dtype=np.uint8)
    if bits == 16 or dist in fsgen.DISTS_WIDE:
        return fsgen.keys_host(dist, bits, n, seed)
    # all-equal wide keys: every digit trivial
    return np.full(n, 0x1234567890ABCDEF & ((1 << bits) - 1), dtype=fsgen.key_dtype(bits))


@pytest.mark.parametrize("bits", [8, 16, 32, 64])
@pytest.mark.parametrize("vb", [0, 4, 8])
def test_clobber_input_matches_oracle(gpu, bits, vb):
    """FS_FLAG_CLOBBER_INPUT: the input arrays are the passes' second
    buffer.  Odd and even numbers of active digits (an even number ends in
    the input and is copied out), all-trivial inputs (a copy) and ragged
    sizes all give the oracle's bytes."""
    ws = fs.Workspace(gpu)
    dists = ("uniform", "equal", "presorted") if bits in (8, 16) else ("uniform", "small20", "hot90", "equal")
    for n in (1, 4097, 3 * 4096 + 17, (1 << 18) + 5):
        for di, dist in enumerate(dists):
            seed = fsgen.seed_for(7, di) + n
            k = _clobber_keys(bits, dist, n, seed)
            if vb:
                v = _vals(n, vb, seed)
                ko, vo = fs.sort_pairs(dev(k), dev(v), workspace=ws, clobber=True)
                ek, ev = oracle.sort(k, v)
                assert np.array_equal(host(vo), ev), (bits, vb, n, dist)
            else:
                ko = fs.sort_keys(dev(k), workspace=ws, clobber=True)
                ek = oracle.sort(k)
            torch.cuda.synchronize()
            assert ws.error_word() == 0
            assert np.array_equal(host(ko), ek), (bits, vb, n, dist)


def test_index_payload_is_stable_permutation(gpu):
    """The configs' payload (original index): invariants pin the result."""
    n = 5 * 4096 + 3
    for dist in fsgen.DISTS_16:
        k = fsgen.keys_host(dist, 16, n, 11)
        ko, vo = fs.sort_pairs(dev(k), dev(fsgen.vals_host(n, 4)))
        check_index_pairs(k, host(ko), host(vo))


def test_empty_and_single(gpu):
    for bits in (16, 32, 64):
        dt = fsgen.key_dtype(bits)
        e = fs.sort_keys(dev(np.zeros(0, dtype=dt)))
        assert e.numel() == 0
        one = fs.sort_keys(dev(np.array([7], dtype=dt)))
        assert host(one).tolist() == [7]
        ko, vo = fs.sort_pairs(dev(np.array([9], dtype=dt)), dev(np.array([3], dtype=np.uint32)))
        assert host(ko).tolist() == [9] and host(vo).tolist() == [3]


def test_unaligned_buffers(gpu):
    """Views that start 2 bytes past a 16-byte boundary exercise the
    unaligned head and tail paths of the vector loads and stores."""
    n = 70001
    for bits in (16, 32, 64):
        k = fsgen.keys_host("uniform", bits, n + 3, 5)
        kd = dev(k)[1:1 + n]
        outbuf = torch.empty(n + 1, dtype=kd.dtype, device=gpu)
        out = fs.sort_keys(kd, out=outbuf[1:])
        assert np.array_equal(host(out), oracle.sort(k[1:1 + n])), bits


def test_unaligned_pair_buffers(gpu):
    """16-bit pair sorts over views that start past a 16-byte boundary:
    the first pass writes the high key bytes into the misaligned output
    buffer and the second pass reads them back as one-byte keys, over many
    8192-key tiles and a ragged tail, with 4- and 8-byte payloads, in
    unsigned and in signed descending order."""
    n = (1 << 20) + 12345
    rng = np.random.default_rng(21)
    k = rng.integers(0, 65536, n + 3).astype(np.uint16)
    for vb in (4, 8):
        v = rng.integers(0, 1 << 31, n + 3).astype(np.uint32 if vb == 4 else np.uint64)
        kd, vd = dev(k)[1:1 + n], dev(v)[1:1 + n]
        kob = torch.empty(n + 1, dtype=kd.dtype, device=gpu)
        vob = torch.empty(n + 1, dtype=vd.dtype, device=gpu)
        for key_type, desc in (("unsigned", False), ("signed", True)):
            ko, vo = fs.sort_pairs(kd, vd, keys_out=kob[1:], vals_out=vob[1:], key_type=key_type,
                                   descending=desc)
            torch.cuda.synchronize()
            ek, ev = oracle.sort_ordered(k[1:1 + n], v[1:1 + n], key_type=key_type, descending=desc)
            assert np.array_equal(host(ko), ek), (vb, key_type)
            assert np.array_equal(host(vo), ev), (vb, key_type)


def test_all_equal_is_a_copy(gpu):
    n = 3 * 4096 + 5
    for bits in (16, 32, 64):
        k = np.full(n, 12345, dtype=fsgen.key_dtype(bits))
        v = np.arange(n, dtype=np.uint64)
        ko, vo = fs.sort_pairs(dev(k), dev(v))
        assert np.array_equal(host(ko), k) and np.array_equal(host(vo), v)


def test_digit_histograms_match_oracle(gpu):
    for bits in (16, 32, 64):
        for dist in fsgen.valid_dists(bits):
            for n in (1, 4097, (1 << 20) + 9):
                k = fsgen.keys_host(dist, bits, n, 3)
                h = host(fs.digit_histograms(dev(k), 8)).astype(np.uint64)
                for j in range(bits // 8):
                    assert np.array_equal(h[j], oracle.histogram(k, 8 * j, 8)), (bits, dist, n, j)
    for dist in fsgen.DISTS_16:
        for n in (1, 4097, (1 << 21) + 9):
            k = fsgen.keys_host(dist, 16, n, 4)
            h = host(fs.digit_histograms(dev(k), 16)).astype(np.uint64)[0]
            assert np.array_equal(h, oracle.histogram(k, 0, 16)), (dist, n)


def test_compressed_counters_wrap_exactly(gpu):
    """All keys in one bin, and two bins sharing a counter word, each far
    past 2^16 per workgroup and past 2^32 in total pairs of words: the
    packed 16-bit counters wrap many times and must still decode exactly."""
    n = (1 << 24) + 5
    a = np.full(n, 0x1234, dtype=np.uint16)
    h = host(fs.digit_histograms(dev(a), 16)).astype(np.uint64)[0]
    assert h[0x1234] == n and h.sum() == n
    b = np.where(np.arange(n) % 3 == 0, 0x4444, 0x4445).astype(np.uint16)
    h = host(fs.digit_histograms(dev(b), 16)).astype(np.uint64)[0]
    assert np.array_equal(h, oracle.histogram(b, 0, 16))
    out = fs.sort_keys(dev(b))
    assert np.array_equal(host(out), np.sort(b))
    # pair sorts build the same compressed histogram in their first read and
    # expand their output keys from it
    idx = np.arange(n, dtype=np.uint32)
    for keys in (a, b):
        ko, vo = fs.sort_pairs(dev(keys), dev(idx))
        ek, ev = oracle.sort(keys, idx)
        assert np.array_equal(host(ko), ek)
        assert np.array_equal(host(vo), ev)


def test_repeatable(gpu):
    n = (1 << 20) + 11
    k = dev(fsgen.keys_host("uniform", 32, n, 21))
    v = dev(fsgen.vals_host(n, 4))
    a = fs.sort_pairs(k, v)
    b = fs.sort_pairs(k, v)
    assert torch.equal(a[0].view(torch.int32), b[0].view(torch.int32))
    assert torch.equal(a[1].view(torch.int32), b[1].view(torch.int32))


def test_invalid_arguments(gpu):
    k = dev(np.arange(100, dtype=np.uint32))
    with pytest.raises(fs.FsError) as e:
        fs.sort_keys(k, out=k)  # in place is an overlap
    assert e.value.status == fs.FS_ERR_INVALID_ARG
    v = dev(np.arange(100, dtype=np.uint32))
    with pytest.raises(fs.FsError):
        fs.sort_pairs(k, v, vals_out=v)


def test_many_offset_levels_and_ragged_tail(gpu):
    """2^28 + 4097 keys: 65537 tiles, so every level of the tile offset scan
    (inside blocks, inside super-blocks, over super-blocks) has several
    entries and the last tile holds one key."""
    n = (1 << 28) + 4097
    seed = fsgen.seed_for(1, 0)
    kd = fsgen.keys_device("uniform", 16, n, seed)
    vd = fsgen.index_device(n, 4)
    ko, vo = fs.sort_pairs(kd, vd)
    k = host(kd)
    ek, ev = oracle.sort(k, np.arange(n, dtype=np.uint32))
    assert np.array_equal(host(ko), ek)
    assert np.array_equal(host(vo), ev)


@pytest.mark.parametrize("vb", [0, 4, 8])
@pytest.mark.parametrize("n", [5 * 4096 + 123, 70001])
def test_u64_runs_of_equal_keys(gpu, n, vb):
    """64-bit keys in runs of 601 equal keys, so that a 4096-key tile holds
    at most 8 digit values and writes four staged slots at a time, with
    runs starting at every offset modulo 4 (four-slot groups that straddle
    a digit boundary) and a ragged last tile: ascending runs (every pass
    sees the runs) and runs of hashed values (the first pass does), in
    ascending unsigned and descending signed order."""
    i = np.arange(n, dtype=np.uint64) // np.uint64(601)
    cases = [i * np.uint64(0x0101010101010101),
             (i + np.uint64(1)) * np.uint64(0x9E3779B97F4A7C15)]
    ws = fs.Workspace(gpu)
    for keys in cases:
        v = _vals(n, vb, n + vb) if vb else None
        for kt, desc in (("unsigned", False), ("signed", True)):
            if vb:
                ko, vo = fs.sort_pairs(dev(keys), dev(v), workspace=ws, key_type=kt, descending=desc)
                ek, ev = oracle.sort_ordered(keys, v, key_type=kt, descending=desc)
                torch.cuda.synchronize()
                assert np.array_equal(host(vo), ev), (n, vb, kt)
            else:
                ko = fs.sort_keys(dev(keys), workspace=ws, key_type=kt, descending=desc)
                ek = oracle.sort_ordered(keys, key_type=kt, descending=desc)
                torch.cuda.synchronize()
            assert ws.error_word() == 0
            assert np.array_equal(host(ko), ek), (n, vb, kt)


@pytest.mark.parametrize("n", [5, 4097, 3 * 8192 + 11, (1 << 20) + 7])
def test_pairs16_keys_far_apart(gpu, n):
    """16-bit pair sorts whose keys take a few values far apart (0, 3,
    40000, 65535): the sorted keys are written from the 2^16-bin prefix
    across long runs of empty bins, within one 8-key chunk and across
    chunks; ascending unsigned and descending signed, 4- and 8-byte
    payloads."""
    rng = np.random.default_rng(n)
    keys = np.array([0, 3, 40000, 65535], dtype=np.uint16)[rng.integers(0, 4, n)]
    ws = fs.Workspace(gpu)
    for vb in (4, 8):
        v = _vals(n, vb, n + vb)
        ko, vo = fs.sort_pairs(dev(keys), dev(v), workspace=ws)
        torch.cuda.synchronize()
        assert ws.error_word() == 0
        ek, ev = oracle.sort(keys, v)
        assert np.array_equal(host(ko), ek) and np.array_equal(host(vo), ev), (n, vb)
        ko, vo = fs.sort_pairs(dev(keys), dev(v), workspace=ws, key_type="signed", descending=True)
        torch.cuda.synchronize()
        ek, ev = oracle.sort_ordered(keys, v, key_type="signed", descending=True)
        assert np.array_equal(host(ko), ek) and np.array_equal(host(vo), ev), (n, vb, "signed desc")


def test_pair_sorts_with_one_active_digit_and_in_a_graph(gpu):
    """16-bit pair sorts above 2^22 keys, whose keys are expanded from the
    2^16-bin prefix and whose second pass sorts by the high key bytes the
    first pass wrote: only the second digit active (the low byte is
    constant, so the high bytes are copied from the input instead), only
    the first (the high byte is constant; that pass is then the last and
    writes only payloads), both; the same in signed descending order (the
    copied bytes are those of the mapped keys), with 8-byte payloads (4096-key
    tiles), and clobbering the input; and the sort captured into a
    hipGraph, replayed twice with the outputs cleared in between."""
    n = (1 << 22) + 3
    rng = np.random.default_rng(5)
    idx = np.arange(n, dtype=np.uint32)
    cases = [(rng.integers(0, 256, n) << 8).astype(np.uint16),        # digit 0 trivial
             (0x3A00 | rng.integers(0, 256, n)).astype(np.uint16),    # digit 1 trivial
             rng.integers(0, 65536, n).astype(np.uint16)]
    for keys in cases:
        ko, vo = fs.sort_pairs(dev(keys), dev(idx))
        torch.cuda.synchronize()
        ek, ev = oracle.sort(keys, idx)
        assert np.array_equal(host(ko), ek)
        assert np.array_equal(host(vo), ev)
        ko, vo = fs.sort_pairs(dev(keys), dev(idx), key_type="signed", descending=True)
        torch.cuda.synchronize()
        ek, ev = oracle.sort_ordered(keys, idx, key_type="signed", descending=True)
        assert np.array_equal(host(ko), ek)
        assert np.array_equal(host(vo), ev)
        idx8 = idx.astype(np.uint64) * np.uint64(0x100000001)
        ko, vo = fs.sort_pairs(dev(keys), dev(idx8))
        torch.cuda.synchronize()
        ek, ev = oracle.sort(keys, idx8)
        assert np.array_equal(host(ko), ek)
        assert np.array_equal(host(vo), ev)
        ko, vo = fs.sort_pairs(dev(keys), dev(idx), clobber=True)
        torch.cuda.synchronize()
        ek, ev = oracle.sort(keys, idx)
        assert np.array_equal(host(ko), ek)
        assert np.array_equal(host(vo), ev)
    keys = cases[2]
    kd, vd = dev(keys), dev(idx)
    ko, vo = torch.empty_like(kd), torch.empty_like(vd)
    ws = fs.Workspace(gpu)
    ws.get(fs.sort_pairs_workspace_bytes(n, 16, 4))
    g = fs.CapturedSort(lambda: fs.sort_pairs(kd, vd, keys_out=ko, vals_out=vo, workspace=ws), gpu)
    ek, ev = oracle.sort(keys, idx)
    for _ in range(2):
        ko.view(torch.int16).zero_()
        vo.view(torch.int32).zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(host(ko), ek)
        assert np.array_equal(host(vo), ev)


def test_sorts_replay_from_a_captured_graph(gpu):
    """A 16-bit keys-only sort and a 16-bit pair sort captured into one HIP
    graph and replayed four times, with other eager sorts and
    synchronisations between replays; the outputs are overwritten before
    every replay and each replay's result must equal the oracle's."""
    n = 3 * (1 << 20) + 77
    k = fsgen.keys_host("zipf", 16, n, fsgen.seed_for(1, 2) + 7)
    v = fsgen.vals_host(n, 4)
    ki, vi = dev(k), dev(v)
    ek = oracle.sort(k)
    pk, pv = oracle.sort(k, v)
    ko, ko2, vo2 = torch.empty_like(ki), torch.empty_like(ki), torch.empty_like(vi)
    ws1, ws2 = fs.Workspace(gpu), fs.Workspace(gpu)
    ws1.get(fs.sort_keys_workspace_bytes(n, 16))
    ws2.get(fs.sort_pairs_workspace_bytes(n, 16, 4))

    def step():
        fs.sort_keys(ki, out=ko, workspace=ws1)
        fs.sort_pairs(ki, vi, keys_out=ko2, vals_out=vo2, workspace=ws2)

    side = torch.cuda.Stream(gpu)
    side.wait_stream(torch.cuda.current_stream(gpu))
    with torch.cuda.stream(side):
        step()
    torch.cuda.current_stream(gpu).wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        step()
    other = dev(fsgen.keys_host("uniform", 16, 100_003, 5))
    for r in range(4):
        for t in (ko, ko2, vo2):
            t.view(torch.uint8).fill_(0xA5)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert ws1.error_word() == 0 and ws2.error_word() == 0, r
        assert np.array_equal(host(ko), ek), r
        assert np.array_equal(host(ko2), pk) and np.array_equal(host(vo2), pv), r
        # eager work of the program between replays
        fs.sort_keys(other)
        torch.cuda.synchronize()
