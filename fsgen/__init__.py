"""Seeded synthetic inputs for the sort (shared by tests, smoke and bench).

This module holds none of the sort's arithmetic: it only draws keys.  Both
the CPU oracle and the HIP path receive the same bytes from here.

Every draw comes from one counter-based generator, the SplitMix64 output
function (Steele, Lea & Flood, "Fast splittable pseudorandom number
generators", OOPSLA 2014): the i-th draw of stream s under seed S is

    z = (S ^ (s * GOLDEN)) + (i + 1) * GOLDEN          (mod 2^64)
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9
    z = (z ^ (z >> 27)) * 0x94D049BB133111EB
    rand64 = z ^ (z >> 31)

It is integer-only, so the numpy implementation here and the device kernel
in gen.hip produce identical bytes.  Non-uniform distributions sample a
host-built table of 64-bit thresholds by counting the thresholds <= x, so
nothing transcendental runs on the device.

Distributions (the paper evaluates uniform keys; the skewed ones stand in
for the skew it leaves to future work):
  16-bit keys: uniform, gaussian (mean 32768, sd 1024, rounded, clamped),
               zipf (s = 1.2 over 65536 ranks, rank r -> key r-1), equal
               (all keys one random value), presorted (floor(i*2^16/n)),
               reverse (65535 - floor(i*2^16/n)).
  32/64-bit:   uniform, small20 (values < 2^20), hot90 (90% of keys from 256
               random hot values, the rest uniform).
"""
import math
import os

import numpy as np

GOLDEN = 0x9E3779B97F4A7C15
MIX1 = 0xBF58476D1CE4E5B9
MIX2 = 0x94D049BB133111EB
BASE_SEED = 0x46534F5254000000  # the bytes "FSORT" shifted up

MASK64 = (1 << 64) - 1

DISTS_16 = ("uniform", "gaussian", "zipf", "equal", "presorted", "reverse")
DISTS_WIDE = ("uniform", "small20", "hot90")
DIST_CODES = {"uniform": 0, "gaussian": 1, "zipf": 2, "equal": 3, "presorted": 4,
              "reverse": 5, "small20": 6, "hot90": 7}

# streams used by the recipes
STREAM_KEYS, STREAM_EQUAL, STREAM_HOT_TABLE, STREAM_HOT_PICK = 0, 1, 2, 3
HOT_THRESHOLD = (9 * (1 << 32)) // 10  # floor(0.9 * 2^32)


def seed_for(config, dist_index):
    """Seed of a workload: base seed + 16 * config + distribution index."""
    return (BASE_SEED + 16 * int(config) + int(dist_index)) & MASK64


def rand64(seed, stream, start, count):
    """Draws start .. start+count-1 of `stream` under `seed` (uint64 array)."""
    s0 = np.uint64((int(seed) ^ ((int(stream) * GOLDEN) & MASK64)) & MASK64)
    i = np.arange(start + 1, start + count + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = s0 + i * np.uint64(GOLDEN)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(MIX1)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(MIX2)
        z = z ^ (z >> np.uint64(31))
    return z


def rand64_scalar(seed, stream, i):
    """One draw, in Python integers (reference for the vector versions)."""
    z = ((seed ^ ((stream * GOLDEN) & MASK64)) + (i + 1) * GOLDEN) & MASK64
    z = ((z ^ (z >> 30)) * MIX1) & MASK64
    z = ((z ^ (z >> 27)) * MIX2) & MASK64
    return z ^ (z >> 31)


def _thresholds_from_cdf(cdf_upto):
    """thr[k] = floor(P(key <= k) * 2^64) for k = 0 .. 65534, as uint64."""
    thr = np.empty(65535, dtype=np.uint64)
    for k in range(65535):
        p = cdf_upto(k)
        t = int(math.floor(p * 2.0 ** 64)) if p < 1.0 else MASK64
        thr[k] = min(max(t, 0), MASK64)
    return thr


_TABLES = {}


def cdf_table(dist):
    """Threshold table of a 16-bit distribution (gaussian or zipf)."""
    if dist in _TABLES:
        return _TABLES[dist]
    if dist == "gaussian":
        mu, sd = 32768.0, 1024.0
        # rounding to nearest: key <= k  iff  x < k + 0.5 ; clamping folds the tails
        tab = _thresholds_from_cdf(
            lambda k: 0.5 * math.erfc(-((k + 0.5 - mu) / sd) / math.sqrt(2.0)))
    elif dist == "zipf":
        s = 1.2
        w = np.arange(1, 65537, dtype=np.float64) ** (-s)
        c = np.cumsum(w)
        c /= c[-1]
        tab = _thresholds_from_cdf(lambda k: float(c[k]))
    else:
        raise ValueError(dist)
    _TABLES[dist] = tab
    return tab


def hot_table(seed, key_bits):
    """The 256 hot values of the hot90 recipe (stream 2)."""
    h = rand64(seed, STREAM_HOT_TABLE, 0, 256)
    if key_bits < 64:
        h = h >> np.uint64(64 - key_bits)
    return h


def key_dtype(key_bits):
    return {16: np.uint16, 32: np.uint32, 64: np.uint64}[key_bits]


def valid_dists(key_bits):
    return DISTS_16 if key_bits == 16 else DISTS_WIDE


def keys_host(dist, key_bits, n, seed):
    """The keys of a workload, drawn on the host with numpy."""
    dt = key_dtype(key_bits)
    if dist not in valid_dists(key_bits):
        raise ValueError(f"{dist} is not a {key_bits}-bit distribution")
    drop = np.uint64(64 - key_bits)
    if dist == "uniform":
        return (rand64(seed, STREAM_KEYS, 0, n) >> drop).astype(dt)
    if dist in ("gaussian", "zipf"):
        x = rand64(seed, STREAM_KEYS, 0, n)
        # key = number of thresholds <= x
        return np.searchsorted(cdf_table(dist), x, side="right").astype(dt)
    if dist == "equal":
        v = rand64_scalar(seed, STREAM_EQUAL, 0) >> (64 - key_bits)
        return np.full(n, v, dtype=dt)
    if dist in ("presorted", "reverse"):
        i = np.arange(n, dtype=np.uint64)
        k = (i << np.uint64(16)) // np.uint64(max(n, 1))
        if dist == "reverse":
            k = np.uint64(65535) - k
        return k.astype(dt)
    if dist == "small20":
        return (rand64(seed, STREAM_KEYS, 0, n) >> np.uint64(44)).astype(dt)
    if dist == "hot90":
        x = rand64(seed, STREAM_KEYS, 0, n) >> drop
        y = rand64(seed, STREAM_HOT_PICK, 0, n)
        hot = hot_table(seed, key_bits)[((y >> np.uint64(8)) & np.uint64(255)).astype(np.int64)]
        pick = (y >> np.uint64(32)) < np.uint64(HOT_THRESHOLD)
        return np.where(pick, hot, x).astype(dt)
    raise ValueError(dist)


def vals_host(n, val_bytes=4, kind="index", seed=0):
    """Payload: the original index (the configs' choice) or random words."""
    dt = np.uint32 if val_bytes == 4 else np.uint64
    if kind == "index":
        return np.arange(n, dtype=dt)
    r = rand64(seed, 9, 0, n)
    return (r >> np.uint64(32)).astype(dt) if val_bytes == 4 else r


# ---------------------------------------------------------------- device side
_dev = None
HERE = os.path.dirname(os.path.abspath(__file__))
DEV_LIB = os.path.join(HERE, "libfsgen.so")


def _load_device():
    global _dev
    if _dev is not None:
        return _dev
    import ctypes
    if not os.path.exists(DEV_LIB):
        raise RuntimeError(f"{DEV_LIB} is not built; run __graft_entry__.build()")
    lib = ctypes.CDLL(DEV_LIB)
    vp, u64, i32 = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int
    lib.fsgen_keys.argtypes = [vp, u64, i32, i32, u64, vp, vp]
    lib.fsgen_keys.restype = i32
    lib.fsgen_index.argtypes = [vp, u64, i32, u64, vp]
    lib.fsgen_index.restype = i32
    _dev = lib
    return lib


def keys_device(dist, key_bits, n, seed, device="cuda", out=None):
    """Same bytes as keys_host(dist, key_bits, n, seed), drawn on the GPU.

    `out` is an optional preallocated torch tensor of n keys.
    """
    import torch
    if dist not in valid_dists(key_bits):
        raise ValueError(f"{dist} is not a {key_bits}-bit distribution")
    tdt = {16: torch.uint16, 32: torch.uint32, 64: torch.uint64}[key_bits]
    if out is None:
        out = torch.empty(n, dtype=tdt, device=device)
    table = None
    if dist in ("gaussian", "zipf"):
        table = torch.from_numpy(cdf_table(dist).view(np.int64)).to(out.device)
    elif dist == "hot90":
        hot = hot_table(seed, key_bits).astype(np.uint64).view(np.int64)
        table = torch.from_numpy(hot).to(out.device)
    lib = _load_device()
    stream = torch.cuda.current_stream(out.device).cuda_stream
    rc = lib.fsgen_keys(out.data_ptr(), n, key_bits, DIST_CODES[dist], seed,
                        table.data_ptr() if table is not None else None, stream)
    if rc != 0:
        raise RuntimeError(f"fsgen_keys failed with code {rc}")
    if table is not None:  # freed only once the stream is past the generator
        table.record_stream(torch.cuda.current_stream(out.device))
    return out


def index_device(n, val_bytes=4, device="cuda", out=None):
    """Payload equal to the original index, written on the GPU."""
    import torch
    tdt = torch.uint32 if val_bytes == 4 else torch.uint64
    if out is None:
        out = torch.empty(n, dtype=tdt, device=device)
    lib = _load_device()
    stream = torch.cuda.current_stream(out.device).cuda_stream
    rc = lib.fsgen_index(out.data_ptr(), n, val_bytes, 0, stream)
    if rc != 0:
        raise RuntimeError(f"fsgen_index failed with code {rc}")
    return out


# ------------------------------------------------------------ segment batches
def lognormal_lengths(count, seed, median=2048.0, sigma=2.0, cap=1 << 22):
    """Segment lengths L = clamp(round(exp(ln median + sigma * z)), 1, cap),
    with z standard normal by the Box-Muller transform of two seeded uniform
    draws (streams 5 and 6)."""
    u1 = (rand64(seed, 5, 0, count) >> np.uint64(11)).astype(np.float64) * 2.0 ** -53
    u2 = (rand64(seed, 6, 0, count) >> np.uint64(11)).astype(np.float64) * 2.0 ** -53
    u1 = np.maximum(u1, 2.0 ** -53)
    z = np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2)
    L = np.rint(np.exp(np.log(median) + sigma * z))
    return np.clip(L, 1, cap).astype(np.int64)


def segment_plan(count, seed, median=2048.0, sigma=2.0, cap=1 << 22):
    """The batched workload: per segment its length, key width (16 for even
    index, 32 for odd) and distribution (uniform or zipf by a seeded coin)."""
    L = lognormal_lengths(count, seed, median, sigma, cap)
    bits = np.where(np.arange(count) % 2 == 0, 16, 32)
    coin = (rand64(seed, 7, 0, count) >> np.uint64(63)).astype(np.int64)
    dist = np.where(coin == 1, "zipf", "uniform")
    return L, bits, dist
