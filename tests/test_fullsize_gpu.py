"""Parity at the full workload sizes, in the launch configuration the
benchmark times (the same entry points on the same device-resident inputs).

The oracle cannot sort these sizes in a test, so every result is checked by
properties that fix the sorted output uniquely, computed with plain PyTorch
ops (nothing from the HIP library), plus sampled positions the oracle
computes one by one:
  * pairs with the index payload (2^31 u16 + u32, 2^31 u32 + u32): the
    payload is a permutation of 0..n-1, keys_out[i] == keys_in[vals_out[i]],
    keys are non-decreasing and equal keys keep increasing indices --
    together these define the stable sort exactly;
  * 16-bit keys only (2^28): non-decreasing, and the 2^16 value counts equal
    those of the input (for 16-bit keys that is the whole multiset);
  * 64-bit keys only (2^32): every output key against the partitioned
    oracle (oracle.partitioned): the input is cut in key order into ranges
    of at most 2^28 keys, each sorted by the oracle's counting sort and
    compared with the output at the offset its key counts fix;
  * sampled positions of the 16-bit sorts against oracle.select over the
    oracle's histogram of the input, and their payloads against the input
    position of that key's occurrence;
  * the batched workload (10^5 log-normal segments, u16/u32, about 1.46e9
    keys, built as the benchmark builds it): every segment against
    torch.sort of (segment id, key) over the whole batch, and a sample of
    segments (the longest ones among them) against the oracle;
  * 2^30 u8 keys with the index payload: the stable-pair properties above,
    plus the 256 value counts of input and output;
  * 2^28 keys of 128 bits: the keys-only result equals the keys of the
    sort with an index payload, and that payload satisfies the stable-pair
    properties over whole 128-bit keys.
"""
import numpy as np
import pytest
import torch

import fsgen
import oracle
from oracle.partitioned import partitioned_sort
import paper_2605_10390_amd as fs

pytestmark = pytest.mark.gpu

CHUNK = 1 << 28
I64_MIN = -(1 << 63)


def as_i64(t):
    """Unsigned keys as int64 values in the same order (16/32-bit: widened;
    64-bit: sign bit flipped)."""
    if t.dtype == torch.uint8:
        return t.to(torch.int64)
    if t.dtype == torch.uint16:
        return t.view(torch.int16).to(torch.int64) & 0xFFFF
    if t.dtype == torch.uint32:
        return t.view(torch.int32).to(torch.int64) & 0xFFFFFFFF
    return t.view(torch.int64) ^ I64_MIN


SIGNED = {torch.uint8: torch.int8, torch.uint16: torch.int16, torch.uint32: torch.int32, torch.uint64: torch.int64}


def bits(t):
    """The same bits as a signed tensor (for equality tests and indexing)."""
    return t.view(SIGNED[t.dtype])


def check_non_decreasing(ko):
    n = ko.numel()
    for a in range(0, n, CHUNK):
        c = as_i64(ko[a:min(n, a + CHUNK + 1)])
        assert bool((c[1:] >= c[:-1]).all()), f"not sorted near {a}"


def check_stable_pairs(ki, ko, vo):
    """vo is a permutation, ko[i] == ki[vo[i]], and equal keys keep order."""
    n = ki.numel()
    seen = torch.zeros(n, dtype=torch.bool, device=ki.device)
    for a in range(0, n, CHUNK):
        b = min(n, a + CHUNK)
        idx = vo[a:b].view(torch.int32).to(torch.int64) & 0xFFFFFFFF
        assert int(idx.max()) < n
        seen[idx] = True
        assert torch.equal(bits(ki)[idx], bits(ko)[a:b]), f"keys_out != keys_in[vals_out] near {a}"
        e = min(n, b + 1)
        k = as_i64(ko[a:e])
        v = vo[a:e].view(torch.int32).to(torch.int64) & 0xFFFFFFFF
        eq = k[1:] == k[:-1]
        assert bool((v[1:][eq] > v[:-1][eq]).all()), f"equal keys out of input order near {a}"
        del idx, k, v, eq
    assert bool(seen.all()), "payload is not a permutation"


def counts16(t, shift):
    out = torch.zeros(65536, dtype=torch.int64, device=t.device)
    for a in range(0, t.numel(), CHUNK):
        c = as_i64(t[a:a + CHUNK])
        if t.dtype == torch.uint64:
            c = c ^ I64_MIN  # back to the raw bits
        # sort-based counting: no atomic contention when few values dominate
        vals, cnt = torch.unique((c >> shift) & 0xFFFF, return_counts=True)
        out.index_add_(0, vals, cnt)
    return out


def sampled_positions(n, count, seed):
    rng = np.random.default_rng(seed)
    return sorted({0, n - 1, *rng.integers(0, n, count).tolist()})


def nth_occurrence(t, value, r):
    """Input position of the r-th (from 0) element of t equal to value."""
    for a in range(0, t.numel(), CHUNK):
        hit = t[a:a + CHUNK] == value
        c = int(hit.sum())
        if r < c:
            return a + int(torch.nonzero(hit).flatten()[r])
        r -= c
    raise AssertionError("fewer occurrences than the rank asks for")


def check_u16_samples(ki_host, ko, vo=None, ki=None, count=6):
    hist = oracle.histogram(ki_host, 0, 16)
    prefix = oracle.exclusive_scan(hist)
    ko_h = ko.cpu().numpy()
    for i in sampled_positions(ko.numel(), count, 5):
        v = oracle.select(hist, i)
        assert int(ko_h[i]) == v, i
        if vo is not None:
            want = nth_occurrence(bits(ki), v if v < 32768 else v - 65536, i - int(prefix[v]))
            assert int(vo[i].view(torch.int32).item()) & 0xFFFFFFFF == want, i


def test_c0_u16_keys_2e28(gpu):
    n = 1 << 28
    ki = fsgen.keys_device("uniform", 16, n, fsgen.seed_for(0, 0), device=gpu)
    ws = fs.Workspace(gpu)
    ko = fs.sort_keys(ki, workspace=ws)
    torch.cuda.synchronize()
    assert ws.error_word() == 0
    check_non_decreasing(ko)
    assert torch.equal(counts16(ki, 0), counts16(ko, 0))
    check_u16_samples(ki.cpu().numpy(), ko)


@pytest.mark.parametrize("dist", fsgen.DISTS_16)
def test_c1_u16_pairs_2e31(gpu, dist):
    n = 1 << 31
    ki = fsgen.keys_device(dist, 16, n, fsgen.seed_for(1, fsgen.DISTS_16.index(dist)), device=gpu)
    vi = fsgen.index_device(n, 4, device=gpu)
    ws = fs.Workspace(gpu)
    ko, vo = fs.sort_pairs(ki, vi, workspace=ws)
    torch.cuda.synchronize()
    assert ws.error_word() == 0
    del vi
    check_stable_pairs(ki, ko, vo)
    check_u16_samples(ki.cpu().numpy(), ko, vo, ki, count=4)


@pytest.mark.parametrize("dist", fsgen.DISTS_WIDE)
def test_c2_u32_pairs_2e31(gpu, dist):
    n = 1 << 31
    ki = fsgen.keys_device(dist, 32, n, fsgen.seed_for(2, fsgen.DISTS_WIDE.index(dist)), device=gpu)
    vi = fsgen.index_device(n, 4, device=gpu)
    ws = fs.Workspace(gpu)
    ko, vo = fs.sort_pairs(ki, vi, workspace=ws)
    torch.cuda.synchronize()
    assert ws.error_word() == 0
    del vi
    check_stable_pairs(ki, ko, vo)


@pytest.mark.parametrize("dist", fsgen.DISTS_WIDE)
def test_c2_u64_keys_2e32(gpu, dist):
    """Every one of the 2^32 output keys against the partitioned oracle:
    the input is cut in key order into ranges of at most 2^28 keys (16-bit
    windows, split again where one bin is larger), each range sorted by
    oracle.sort and compared with the output at its offset."""
    n = 1 << 32
    ki = fsgen.keys_device(dist, 64, n, fsgen.seed_for(2, fsgen.DISTS_WIDE.index(dist)), device=gpu)
    ws = fs.Workspace(gpu)
    ko = fs.sort_keys(ki, workspace=ws)
    torch.cuda.synchronize()
    assert ws.error_word() == 0
    del ws
    kh = ki.cpu().numpy()
    del ki
    compared = 0
    for off, expected in partitioned_sort(kh, 64, 1 << 28, threads=16):
        got = ko[off:off + expected.size].cpu().numpy()
        assert np.array_equal(got, expected), (dist, off, expected.size)
        compared += expected.size
    assert compared == n


def test_c3_segmented_batch_full(gpu):
    from bench import build_c3
    batch, desc, pools, L = build_c3(gpu)
    ws = batch.run()
    torch.cuda.synchronize()
    assert ws.error_word() == 0
    for (b, dname), (g, out, sel, offs) in pools.items():
        lens = torch.from_numpy(L[sel].astype(np.int64)).to(gpu)
        seg = torch.repeat_interleave(torch.arange(sel.size, device=gpu, dtype=torch.int64), lens)
        want = torch.sort((seg << b) | as_i64(g)).values & ((1 << b) - 1)
        assert torch.equal(want, as_i64(out)), (b, dname)
        del seg, want
    rng = np.random.default_rng(3)
    order = np.argsort(L)[::-1]
    sample = set(order[:3].tolist()) | set(rng.choice(L.size, 40, replace=False).tolist())
    for s in sorted(sample):
        b = int(desc["key_bits"][s])
        g, out, sel, offs = next(v for (bb, _), v in pools.items() if bb == b and s in set(v[2].tolist()))
        j = int(np.flatnonzero(sel == s)[0])
        a, n = int(offs[j]), int(L[s])
        k = g[a:a + n].cpu().numpy()
        assert np.array_equal(out[a:a + n].cpu().numpy(), oracle.sort(k)), s


def test_pairs_beyond_2e32_elements(gpu):
    """2^32 + 4099 u16 keys with a u64 index payload: positions, counts and
    offsets pass 2^32 (64-bit throughout).  Checked by the properties that
    fix a stable sort: non-decreasing keys, the payload a permutation of
    0..n-1, keys_out[i] == keys_in[vals_out[i]], equal keys in input order."""
    n = (1 << 32) + 4099
    ki = fsgen.keys_device("zipf", 16, n, fsgen.seed_for(1, 2) + 1, device=gpu)
    vi = fsgen.index_device(n, 8, device=gpu)
    ws = fs.Workspace(gpu)
    ko, vo = fs.sort_pairs(ki, vi, workspace=ws)
    torch.cuda.synchronize()
    assert ws.error_word() == 0
    del vi, ws
    torch.cuda.empty_cache()
    seen = torch.zeros(n, dtype=torch.bool, device=gpu)
    for a in range(0, n, CHUNK):
        b = min(n, a + CHUNK)
        idx = vo[a:b].view(torch.int64)
        assert int(idx.min()) >= 0 and int(idx.max()) < n
        seen[idx] = True
        assert torch.equal(bits(ki)[idx], bits(ko)[a:b]), a
        e = min(n, b + 1)
        k = as_i64(ko[a:e])
        v = vo[a:e].view(torch.int64)
        assert bool((k[1:] >= k[:-1]).all()), a
        eq = k[1:] == k[:-1]
        assert bool((v[1:][eq] > v[:-1][eq]).all()), a
        del idx, k, v, eq
    assert bool(seen.all())


def test_u8_pairs_2e30(gpu):
    """The 8-bit workload as the benchmark builds it: the high byte of the
    uniform 16-bit recipe, with the index payload."""
    n = 1 << 30
    k16 = fsgen.keys_device("uniform", 16, n, fsgen.seed_for(8, 0), device=gpu)
    ki = ((k16.view(torch.int16).to(torch.int32) >> 8) & 0xFF).to(torch.uint8)
    del k16
    vi = fsgen.index_device(n, 4, device=gpu)
    ws = fs.Workspace(gpu)
    ko, vo = fs.sort_pairs(ki, vi, workspace=ws)
    torch.cuda.synchronize()
    assert ws.error_word() == 0
    del vi
    check_stable_pairs(ki, ko, vo)
    cin = torch.zeros(256, dtype=torch.int64, device=gpu)
    cout = torch.zeros(256, dtype=torch.int64, device=gpu)
    for a in range(0, n, CHUNK):
        for t, c in ((ki, cin), (ko, cout)):
            vals, cnt = torch.unique(t[a:a + CHUNK].to(torch.int64), return_counts=True)
            c.index_add_(0, vals, cnt)
    assert torch.equal(cin, cout)


def test_wide128_keys_2e28(gpu):
    """2^28 keys of two uniform 64-bit words, as the benchmark builds them."""
    n, words = 1 << 28, 2
    keys = fsgen.keys_device("uniform", 64, n * words, fsgen.seed_for(9, 0), device=gpu).view(torch.int64)
    keys = keys.view(n, words)
    ws = fs.Workspace(gpu)
    ko = fs.sort_wide(keys, workspace=ws)
    idx = fsgen.index_device(n, 4, device=gpu)
    ko2, vo = fs.sort_wide(keys, vals=idx, workspace=ws)
    torch.cuda.synchronize()
    assert ws.error_word() == 0
    del idx
    assert torch.equal(ko, ko2), "keys-only result differs from the pair sort's keys"
    del ko2
    seen = torch.zeros(n, dtype=torch.bool, device=gpu)
    flat = keys.view(-1)  # word w of key i at 2i + w: rows are gathered as 1-D words
    for a in range(0, n, CHUNK // 4):
        b = min(n, a + CHUNK // 4)
        e = min(n, b + 1)
        idx = vo[a:b].view(torch.int32).to(torch.int64) & 0xFFFFFFFF
        seen[idx] = True
        for w in range(words):
            assert torch.equal(flat[idx * words + w], ko[a:b, w].contiguous()), (a, w)
        hi = ko[a:e, 1] ^ I64_MIN
        lo = ko[a:e, 0] ^ I64_MIN
        v = vo[a:e].view(torch.int32).to(torch.int64) & 0xFFFFFFFF
        gt = (hi[1:] > hi[:-1]) | ((hi[1:] == hi[:-1]) & (lo[1:] > lo[:-1]))
        eq = (hi[1:] == hi[:-1]) & (lo[1:] == lo[:-1])
        assert bool((gt | eq).all()), f"not sorted near {a}"
        assert bool((v[1:][eq] > v[:-1][eq]).all()), f"equal keys out of input order near {a}"
    assert bool(seen.all()), "payload is not a permutation"
