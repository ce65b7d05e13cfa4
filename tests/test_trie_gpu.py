"""GPU parity of the sparse-trie plan (32- and 64-bit keys, n far below 2^p):
the top ceil(log2 n) bits sorted by the window passes, every run of equal
window prefix sorted by its trailing bits in the fixup, and the full LSD
fallback when a run is too long for it.  Every result equals the oracle's,
byte for byte.  The plan words in the workspace say which path ran, so each
case checks that it exercised the path it is about.
"""
import numpy as np
import pytest
import torch

import fsgen
import oracle
import paper_2605_10390_amd as fs
from tests.checks import check_index_pairs

pytestmark = pytest.mark.gpu

TRIE_MIN = 1 << 22
PLAN_BYTE = 256           # the plan follows the 256-byte error-word block
K_TRIE, K_COND_SLOT = 66, 8


def plan_words(ws):
    return ws.buf[PLAN_BYTE:PLAN_BYTE + 72 * 4].view(torch.int32).cpu().numpy()


def path_taken(ws):
    p = plan_words(ws)
    if not p[K_TRIE]:
        return "lsd"
    return "fallback" if p[4 * K_COND_SLOT] else "trie"


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def sparse_u64(n, seed):
    return fsgen.keys_host("uniform", 64, n, seed)


@pytest.mark.parametrize("n", [TRIE_MIN + 13, (1 << 24) + 3])
def test_u64_keys_trie_window_and_fixup(gpu, n):
    k = sparse_u64(n, 41 + n)
    ws = fs.Workspace(gpu)
    out = fs.sort_keys(dev(k), workspace=ws)
    torch.cuda.synchronize()
    assert ws.error_word() == 0
    assert path_taken(ws) == "trie"
    assert np.array_equal(out.cpu().numpy(), oracle.sort(k))


@pytest.mark.parametrize("vb", [4, 8])
def test_u32_pairs_trie_is_stable(gpu, vb):
    n = TRIE_MIN + 77
    k = fsgen.keys_host("uniform", 32, n, 5)
    k[::2000] = k[3]                       # a run of ~2100 equal keys (+ rare neighbours): sorted in LDS
    v = np.arange(n, dtype=np.uint32 if vb == 4 else np.uint64)
    ws = fs.Workspace(gpu)
    ko, vo = fs.sort_pairs(dev(k), dev(v), workspace=ws)
    torch.cuda.synchronize()
    assert ws.error_word() == 0
    assert path_taken(ws) == "trie"
    ek, ev = oracle.sort(k, v)
    assert np.array_equal(ko.cpu().numpy(), ek) and np.array_equal(vo.cpu().numpy(), ev)


@pytest.mark.parametrize("vals", [False, True])
def test_long_unsorted_runs_take_the_fallback(gpu, vals):
    # digits 5, 6 and 7 each uniform over 256 values (no heavy bin) but all
    # equal to one another, so the window bits take only 256 values: runs of
    # about 16K keys with random low bits, which the fixup must hand to the
    # full LSD
    n = TRIE_MIN + 1001
    rng = np.random.default_rng(9)
    x = rng.integers(0, 256, n, dtype=np.uint64)
    k = (x << np.uint64(56)) | (x << np.uint64(48)) | (x << np.uint64(40)) | rng.integers(0, 1 << 40, n, dtype=np.uint64)
    k[5::400] = k[5]                       # equal keys across the array (stability)
    ws = fs.Workspace(gpu)
    if vals:
        v = np.arange(n, dtype=np.uint32)
        ko, vo = fs.sort_pairs(dev(k), dev(v), workspace=ws)
    else:
        ko = fs.sort_keys(dev(k), workspace=ws)
    torch.cuda.synchronize()
    assert ws.error_word() == 0
    assert path_taken(ws) == "fallback"
    if vals:
        check_index_pairs(k, ko.cpu().numpy(), vo.cpu().numpy())
        ek, ev = oracle.sort(k, v)
        assert np.array_equal(vo.cpu().numpy(), ev)
    else:
        assert np.array_equal(ko.cpu().numpy(), oracle.sort(k))


def test_skewed_keys_keep_the_plain_plan(gpu):
    # 90% of keys from 256 hot values: heavy digit bins, so the plan keeps
    # the plain LSD instead of a window whose runs would be long
    n = TRIE_MIN + 5
    k = fsgen.keys_host("hot90", 64, n, 17)
    ws = fs.Workspace(gpu)
    out = fs.sort_keys(dev(k), workspace=ws)
    torch.cuda.synchronize()
    assert path_taken(ws) == "lsd"
    assert np.array_equal(out.cpu().numpy(), oracle.sort(k))


def test_runs_of_equal_keys_need_no_fallback(gpu):
    # long runs made of one repeated key are in order already
    n = TRIE_MIN + 9
    k = sparse_u64(n, 99)
    k[::300] = k[1]
    ws = fs.Workspace(gpu)
    out = fs.sort_keys(dev(k), workspace=ws)
    torch.cuda.synchronize()
    assert path_taken(ws) in ("trie", "lsd")
    assert np.array_equal(out.cpu().numpy(), oracle.sort(k))


@pytest.mark.parametrize("bits,n", [(64, (1 << 24) + 9), (32, TRIE_MIN + 3)])
def test_clobber_both_window_parities(gpu, bits, n):
    # 2^24+ keys: a window of four digits, an even chain that ends in the
    # clobbered input and is copied out; 2^22+: three digits, odd
    k = fsgen.keys_host("uniform", bits, n, 23)
    ws = fs.Workspace(gpu)
    out = fs.sort_keys(dev(k), workspace=ws, clobber=True)
    torch.cuda.synchronize()
    assert path_taken(ws) == "trie"
    assert np.array_equal(out.cpu().numpy(), oracle.sort(k))


@pytest.mark.parametrize("key_type,desc", [("signed", False), ("float", True), ("unsigned", True)])
def test_trie_in_every_order(gpu, key_type, desc):
    n = TRIE_MIN + 31
    k = sparse_u64(n, 77)
    v = np.arange(n, dtype=np.uint32)
    ws = fs.Workspace(gpu)
    ko, vo = fs.sort_pairs(dev(k), dev(v), workspace=ws, key_type=key_type, descending=desc)
    torch.cuda.synchronize()
    assert ws.error_word() == 0
    assert path_taken(ws) == "trie"
    ek, ev = oracle.sort_ordered(k, v, key_type=key_type, descending=desc)
    assert np.array_equal(ko.cpu().numpy(), ek) and np.array_equal(vo.cpu().numpy(), ev)


def test_small_sorts_keep_the_plain_plan(gpu):
    n = TRIE_MIN - 1
    k = sparse_u64(n, 3)
    ws = fs.Workspace(gpu)
    out = fs.sort_keys(dev(k), workspace=ws)
    torch.cuda.synchronize()
    assert path_taken(ws) == "lsd"
    assert np.array_equal(out.cpu().numpy(), oracle.sort(k))


@pytest.mark.parametrize("vals", [False, True])
def test_medium_runs_sorted_in_lds(gpu, vals):
    # the window bits take 8192 values (each digit still close to uniform),
    # so runs hold about 500 keys in random order: too long for one thread,
    # short enough for one workgroup's LDS, so no fallback
    n = TRIE_MIN + 333
    rng = np.random.default_rng(12)
    tops = rng.integers(0, 1 << 24, 8192, dtype=np.uint64)
    k = (tops[rng.integers(0, 8192, n)] << np.uint64(40)) | rng.integers(0, 1 << 40, n, dtype=np.uint64)
    k[7::2000] = k[7]                      # repeated keys inside one run (stability)
    ws = fs.Workspace(gpu)
    if vals:
        v = np.arange(n, dtype=np.uint64)
        ko, vo = fs.sort_pairs(dev(k), dev(v), workspace=ws)
    else:
        ko = fs.sort_keys(dev(k), workspace=ws)
    torch.cuda.synchronize()
    assert ws.error_word() == 0
    assert path_taken(ws) == "trie"
    if vals:
        ek, ev = oracle.sort(k, v)
        assert np.array_equal(ko.cpu().numpy(), ek) and np.array_equal(vo.cpu().numpy(), ev)
    else:
        assert np.array_equal(ko.cpu().numpy(), oracle.sort(k))
