"""Python binding of libfsort.so, the MI355X compressed-histogram radix sort.

Argument marshalling only: every step of a sort runs in the HIP kernels
behind include/fs_sort.h.  PyTorch supplies device memory and the current
stream.  There is no CPU fallback: if the HIP library is missing, every call
raises.

Keys are 16/32/64-bit integers or floats; values are 4- or 8-byte words.
Results are stable (equal keys keep their input order).  The key order
follows the dtype unless `key_type` says otherwise: unsigned dtypes sort as
unsigned integers, signed dtypes as two's-complement integers, floating
dtypes in IEEE 754 totalOrder (-NaN < -inf < ... < -0 < +0 < ... < +inf <
+NaN); `descending=True` reverses the order.
"""
import ctypes
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfsort.so")

FS_OK, FS_ERR_INVALID_ARG, FS_ERR_UNSUPPORTED, FS_ERR_WORKSPACE_TOO_SMALL, FS_ERR_DEVICE = range(5)

_KEY_BITS = {torch.uint8: 8, torch.int8: 8, torch.uint16: 16, torch.int16: 16, torch.uint32: 32, torch.int32: 32,
             torch.uint64: 64, torch.int64: 64, torch.float16: 16, torch.bfloat16: 16,
             torch.float32: 32, torch.float64: 64}
FS_FLAG_NONE, FS_FLAG_CLOBBER_INPUT, FS_FLAG_SIGNED, FS_FLAG_FLOAT, FS_FLAG_DESCENDING = 0, 1, 2, 4, 8
_TYPE_FLAGS = {"unsigned": FS_FLAG_NONE, "signed": FS_FLAG_SIGNED, "float": FS_FLAG_FLOAT}
_VAL_BYTES = {torch.uint32: 4, torch.int32: 4, torch.float32: 4, torch.uint64: 8,
              torch.int64: 8, torch.float64: 8}

_lib = None


class FsError(RuntimeError):
    def __init__(self, status, what):
        super().__init__(f"{what}: {status_string(status)} ({status})")
        self.status = status


def lib():
    """The loaded HIP library (raises when it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build(); "
                           "there is no CPU fallback")
    L = ctypes.CDLL(LIB_PATH)
    vp, u64, i32, u32 = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int, ctypes.c_uint32
    sz = ctypes.POINTER(ctypes.c_size_t)
    L.fs_sort_keys.argtypes = [vp, vp, u64, i32, ctypes.c_uint, vp, sz, vp]
    L.fs_sort_keys.restype = i32
    L.fs_sort_keys_noalloc.argtypes = [vp, vp, u64, i32, ctypes.c_uint, vp, vp]
    L.fs_sort_keys_noalloc.restype = i32
    L.fs_sort_pairs.argtypes = [vp, vp, vp, vp, u64, i32, i32, ctypes.c_uint, vp, sz, vp]
    L.fs_sort_pairs.restype = i32
    L.fs_digit_histograms.argtypes = [vp, u64, i32, i32, vp, vp, sz, vp]
    L.fs_digit_histograms.restype = i32
    L.fs_sort_segmented.argtypes = [vp, u32, u64, u64, ctypes.c_uint, vp, sz, vp]
    L.fs_sort_segmented.restype = i32
    tp = ctypes.POINTER(SegTuning)
    L.fs_sort_segmented_tuned.argtypes = [vp, u32, u64, u64, ctypes.c_uint, tp, vp, sz, vp]
    L.fs_sort_segmented_tuned.restype = i32
    for name in ("fs_segmented_default_tuning", "fs_set_segmented_tuning", "fs_get_segmented_tuning"):
        getattr(L, name).argtypes = [tp]
        getattr(L, name).restype = i32
    L.fs_profile_enable.argtypes = [i32]
    L.fs_profile_enable.restype = i32
    L.fs_profile_read.argtypes = [i32, ctypes.POINTER(u64), ctypes.POINTER(u64),
                                  ctypes.POINTER(ctypes.c_double)]
    L.fs_profile_read.restype = i32
    L.fs_sort_keys_wide.argtypes = [vp, vp, u64, i32, ctypes.c_uint, vp, sz, vp]
    L.fs_sort_keys_wide.restype = i32
    L.fs_sort_pairs_wide.argtypes = [vp, vp, vp, vp, u64, i32, i32, ctypes.c_uint, vp, sz, vp]
    L.fs_sort_pairs_wide.restype = i32
    L.fs_hist16_accumulate.argtypes = [vp, u64, ctypes.c_uint, vp, vp, sz, vp]
    L.fs_hist16_accumulate.restype = i32
    L.fs_hist16_prefix.argtypes = [vp, vp, vp]
    L.fs_hist16_prefix.restype = i32
    L.fs_expand16.argtypes = [vp, u64, u64, ctypes.c_uint, vp, vp]
    L.fs_expand16.restype = i32
    L.fs_sort16_host.argtypes = [vp, vp, u64, u64, ctypes.c_uint, vp, sz, vp, vp]
    L.fs_sort16_host.restype = i32
    L.fs_sort_host.argtypes = [vp, vp, u64, i32, u64, u64, ctypes.c_uint, vp, sz, vp, vp]
    L.fs_sort_host.restype = i32
    L.fs_status_string.argtypes = [i32]
    L.fs_status_string.restype = ctypes.c_char_p
    _lib = L
    return L


def status_string(status):
    return lib().fs_status_string(int(status)).decode()


def _stream(t):
    return ctypes.c_void_p(torch.cuda.current_stream(t.device).cuda_stream)


def _check_dev(*ts):
    for t in ts:
        if not t.is_cuda:
            raise ValueError("tensors must live on the GPU (no CPU fallback)")
        if not t.is_contiguous():
            raise ValueError("tensors must be contiguous")


def _key_bits(keys):
    if keys.dtype not in _KEY_BITS:
        raise TypeError(f"unsupported key dtype {keys.dtype}")
    return _KEY_BITS[keys.dtype]


def order_flags(keys, key_type=None, descending=False):
    """fs_sort flags for a key tensor: key_type None follows the dtype."""
    if key_type is None:
        if keys.dtype in (torch.int8, torch.int16, torch.int32, torch.int64):
            key_type = "signed"
        elif keys.dtype.is_floating_point:
            key_type = "float"
        else:
            key_type = "unsigned"
    if key_type not in _TYPE_FLAGS:
        raise ValueError(f"key_type must be one of {sorted(_TYPE_FLAGS)}, not {key_type!r}")
    return _TYPE_FLAGS[key_type] | (FS_FLAG_DESCENDING if descending else 0)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None and t.numel() else ctypes.c_void_p(None)


class Workspace:
    """Reusable device workspace (grows on demand)."""

    def __init__(self, device="cuda"):
        self.device = torch.device(device)
        self.buf = None

    def get(self, nbytes):
        nbytes = max(int(nbytes), 256)
        if self.buf is None or self.buf.numel() < nbytes:
            self.buf = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        return self.buf

    def error_word(self):
        """Device error word of the last call (0 = ok); synchronises."""
        if self.buf is None:
            return 0
        return int(self.buf[:4].view(torch.int32).item())


def sort_keys_workspace_bytes(n, key_bits, flags=FS_FLAG_NONE):
    size = ctypes.c_size_t(0)
    st = lib().fs_sort_keys(None, None, int(n), int(key_bits), int(flags), None, ctypes.byref(size), None)
    if st != FS_OK:
        raise FsError(st, "fs_sort_keys (workspace query)")
    return size.value


def sort_pairs_workspace_bytes(n, key_bits, val_bytes, flags=FS_FLAG_NONE):
    size = ctypes.c_size_t(0)
    st = lib().fs_sort_pairs(None, None, None, None, int(n), int(key_bits), int(val_bytes), int(flags),
                             None, ctypes.byref(size), None)
    if st != FS_OK:
        raise FsError(st, "fs_sort_pairs (workspace query)")
    return size.value


def sort_keys(keys, out=None, workspace=None, key_type=None, descending=False, clobber=False):
    """Stable sort of a 1-D key tensor (returns `out`); order per order_flags.
    clobber=True lets the sort overwrite `keys` (FS_FLAG_CLOBBER_INPUT: no
    temporary copy in the workspace)."""
    _check_dev(keys)
    bits = _key_bits(keys)
    n = keys.numel()
    if out is None:
        out = torch.empty_like(keys)
    _check_dev(out)
    flags = order_flags(keys, key_type, descending) | (FS_FLAG_CLOBBER_INPUT if clobber else 0)
    ws = workspace or Workspace(keys.device)
    need = sort_keys_workspace_bytes(n, bits, flags)
    buf = ws.get(need)
    size = ctypes.c_size_t(buf.numel())
    st = lib().fs_sort_keys(_ptr(keys), _ptr(out), n, bits, flags, _ptr(buf), ctypes.byref(size), _stream(keys))
    if st != FS_OK:
        raise FsError(st, "fs_sort_keys")
    return out


NOALLOC_SCRATCH_BYTES = 64 << 20  # FS_NOALLOC_SCRATCH_BYTES


def sort_keys_noalloc(keys, out, err_out=None, key_type=None, descending=False, clobber=False):
    """sort_keys through fs_sort_keys_noalloc: the library's static per-GPU
    scratch array is the workspace, so the call allocates nothing (the
    caller passes `out`, and optionally `err_out`, a one-element int32/uint32
    device tensor that receives the call's error word).  Calls that overlap
    on one GPU race on that array."""
    _check_dev(keys, out)
    if err_out is not None:
        _check_dev(err_out)
        if err_out.element_size() != 4 or err_out.numel() < 1:
            raise ValueError("err_out must hold one 32-bit word")
    bits = _key_bits(keys)
    flags = order_flags(keys, key_type, descending) | (FS_FLAG_CLOBBER_INPUT if clobber else 0)
    st = lib().fs_sort_keys_noalloc(_ptr(keys), _ptr(out), keys.numel(), bits, flags,
                                    _ptr(err_out), _stream(keys))
    if st != FS_OK:
        raise FsError(st, "fs_sort_keys_noalloc")
    return out


def sort_pairs(keys, vals, keys_out=None, vals_out=None, workspace=None, key_type=None,
               descending=False, clobber=False):
    """Stable sort of (key, value) pairs; returns (keys, values); order per
    order_flags.  clobber=True lets the sort overwrite `keys` and `vals`."""
    _check_dev(keys, vals)
    bits = _key_bits(keys)
    if vals.dtype not in _VAL_BYTES:
        raise TypeError(f"unsupported value dtype {vals.dtype}")
    vb = _VAL_BYTES[vals.dtype]
    n = keys.numel()
    if vals.numel() != n:
        raise ValueError("keys and values differ in length")
    keys_out = torch.empty_like(keys) if keys_out is None else keys_out
    vals_out = torch.empty_like(vals) if vals_out is None else vals_out
    _check_dev(keys_out, vals_out)
    flags = order_flags(keys, key_type, descending) | (FS_FLAG_CLOBBER_INPUT if clobber else 0)
    ws = workspace or Workspace(keys.device)
    buf = ws.get(sort_pairs_workspace_bytes(n, bits, vb, flags))
    size = ctypes.c_size_t(buf.numel())
    st = lib().fs_sort_pairs(_ptr(keys), _ptr(keys_out), _ptr(vals), _ptr(vals_out), n, bits, vb,
                             flags, _ptr(buf), ctypes.byref(size), _stream(keys))
    if st != FS_OK:
        raise FsError(st, "fs_sort_pairs")
    return keys_out, vals_out


def digit_histograms(keys, digit_bits=8, workspace=None):
    """Counts of every digit value: int64 tensor [key_bits/digit_bits, 2**digit_bits]
    (uint64 counts; they never reach 2^63)."""
    _check_dev(keys)
    bits = _key_bits(keys)
    n = keys.numel()
    digits = bits // digit_bits
    out = torch.empty(digits, 1 << digit_bits, dtype=torch.int64, device=keys.device)
    size = ctypes.c_size_t(0)
    L = lib()
    st = L.fs_digit_histograms(None, n, bits, digit_bits, None, None, ctypes.byref(size), None)
    if st != FS_OK:
        raise FsError(st, "fs_digit_histograms (workspace query)")
    ws = workspace or Workspace(keys.device)
    buf = ws.get(size.value)
    size = ctypes.c_size_t(buf.numel())
    st = L.fs_digit_histograms(_ptr(keys), n, bits, digit_bits, _ptr(out), _ptr(buf),
                               ctypes.byref(size), _stream(keys))
    if st != FS_OK:
        raise FsError(st, "fs_digit_histograms")
    return out


def sort_wide(keys, vals=None, keys_out=None, vals_out=None, workspace=None, key_type="unsigned",
              descending=False):
    """Stable sort of keys wider than 64 bits: `keys` is an (n, W) tensor of
    64-bit words (int64 or uint64), word 0 the least significant.  Returns
    keys_out, or (keys_out, vals_out) when `vals` is given.  key_type is
    "unsigned", "signed" (two's complement over the whole width) or "float"
    (sign-magnitude over the whole width)."""
    if keys.dim() != 2 or keys.dtype not in (torch.int64, torch.uint64):
        raise ValueError("keys must be an (n, words) tensor of 64-bit words")
    _check_dev(keys)
    n, words = keys.shape
    if key_type not in _TYPE_FLAGS:
        raise ValueError(f"key_type must be one of {sorted(_TYPE_FLAGS)}, not {key_type!r}")
    flags = _TYPE_FLAGS[key_type] | (FS_FLAG_DESCENDING if descending else 0)
    keys_out = torch.empty_like(keys) if keys_out is None else keys_out
    _check_dev(keys_out)
    L = lib()
    size = ctypes.c_size_t(0)
    vb = 0
    if vals is not None:
        _check_dev(vals)
        if vals.dtype not in _VAL_BYTES or vals.numel() != n:
            raise ValueError("vals must hold one 4- or 8-byte value per key")
        vb = _VAL_BYTES[vals.dtype]
        vals_out = torch.empty_like(vals) if vals_out is None else vals_out
        _check_dev(vals_out)
        st = L.fs_sort_pairs_wide(None, None, None, None, n, words, vb, flags, None, ctypes.byref(size), None)
    else:
        st = L.fs_sort_keys_wide(None, None, n, words, flags, None, ctypes.byref(size), None)
    if st != FS_OK:
        raise FsError(st, "fs_sort_*_wide (workspace query)")
    ws = workspace or Workspace(keys.device)
    buf = ws.get(size.value)
    size = ctypes.c_size_t(buf.numel())
    if vals is not None:
        st = L.fs_sort_pairs_wide(_ptr(keys), _ptr(keys_out), _ptr(vals), _ptr(vals_out), n, words, vb, flags,
                                  _ptr(buf), ctypes.byref(size), _stream(keys))
        if st != FS_OK:
            raise FsError(st, "fs_sort_pairs_wide")
        return keys_out, vals_out
    st = L.fs_sort_keys_wide(_ptr(keys), _ptr(keys_out), n, words, flags, _ptr(buf), ctypes.byref(size),
                             _stream(keys))
    if st != FS_OK:
        raise FsError(st, "fs_sort_keys_wide")
    return keys_out


# ------------------------------------------------------------- segmented sort
import numpy as _np

SEGMENT_DTYPE = _np.dtype([("keys_in", _np.uint64), ("keys_out", _np.uint64),
                           ("vals_in", _np.uint64), ("vals_out", _np.uint64),
                           ("n", _np.uint64), ("key_bits", _np.uint32), ("val_bytes", _np.uint32)])


class SegTuning(ctypes.Structure):
    """fs_seg_tuning: per-bin launch choices of fs_sort_segmented (digit
    width via the 16-bit-digit bin, tile size, workgroups per CU)."""
    _fields_ = [("small_max_keys", ctypes.c_uint32 * 3), ("expand16_min_keys", ctypes.c_uint32),
                ("expand16_split_keys", ctypes.c_uint32), ("expand16_wgs_per_cu", ctypes.c_uint32),
                ("large_wg_max_keys", ctypes.c_uint32),
                ("tile_items", ctypes.c_uint32), ("tile_threads", ctypes.c_uint32),
                ("large_wgs_per_cu", ctypes.c_uint32),
                ("small_wgs_per_cu", ctypes.c_uint32)]

    FIELDS = ("small_max_keys", "expand16_min_keys", "expand16_split_keys", "expand16_wgs_per_cu",
              "large_wg_max_keys",
              "tile_items", "tile_threads", "large_wgs_per_cu", "small_wgs_per_cu")

    def as_dict(self):
        d = {f: getattr(self, f) for f in self.FIELDS}
        d["small_max_keys"] = list(self.small_max_keys)
        return d

    @classmethod
    def from_dict(cls, d):
        t = cls()
        for f in cls.FIELDS:
            if f == "small_max_keys":
                t.small_max_keys[:] = [int(v) for v in d[f]]
            else:
                setattr(t, f, int(d[f]))
        return t

    def copy(self):
        return SegTuning.from_dict(self.as_dict())


def default_tuning():
    t = SegTuning()
    st = lib().fs_segmented_default_tuning(ctypes.byref(t))
    if st != FS_OK:
        raise FsError(st, "fs_segmented_default_tuning")
    return t


def get_tuning():
    t = SegTuning()
    st = lib().fs_get_segmented_tuning(ctypes.byref(t))
    if st != FS_OK:
        raise FsError(st, "fs_get_segmented_tuning")
    return t


def set_tuning(t):
    """Set the process-wide tuning used by fs_sort_segmented (None = defaults)."""
    st = lib().fs_set_segmented_tuning(ctypes.byref(t) if t is not None else None)
    if st != FS_OK:
        raise FsError(st, "fs_set_segmented_tuning")


def sort_segmented_workspace_bytes(count, total_keys, max_segment_keys):
    size = ctypes.c_size_t(0)
    st = lib().fs_sort_segmented(None, int(count), int(total_keys), int(max_segment_keys), 0, None,
                                 ctypes.byref(size), None)
    if st != FS_OK:
        raise FsError(st, "fs_sort_segmented (workspace query)")
    return size.value


class SegmentBatch:
    """A device-resident array of fs_segment descriptors.

    `segments` is a sequence of (keys_in, keys_out, vals_in, vals_out)
    tuples of GPU tensors (vals may be None).  The descriptors are built on
    the host once and copied to the device; `run()` sorts every segment with
    one fs_sort_segmented call.
    """

    def __init__(self, segments, device="cuda"):
        m = len(segments)
        desc = _np.zeros(m, dtype=SEGMENT_DTYPE)
        total, biggest = 0, 0
        for i, (ki, ko, vi, vo) in enumerate(segments):
            n = ki.numel()
            desc[i] = (ki.data_ptr() if n else 0, ko.data_ptr() if n else 0,
                       vi.data_ptr() if vi is not None and n else 0,
                       vo.data_ptr() if vo is not None and n else 0, n, _key_bits(ki),
                       _VAL_BYTES[vi.dtype] if vi is not None else 0)
            total += n
            biggest = max(biggest, n)
        self._keep = segments
        self.from_descriptors(desc, total, biggest, device)

    @classmethod
    def from_array(cls, desc, total_keys, max_segment_keys, device="cuda", keep=None):
        self = cls.__new__(cls)
        self._keep = keep
        self.from_descriptors(desc, total_keys, max_segment_keys, device)
        return self

    def from_descriptors(self, desc, total_keys, max_segment_keys, device):
        self.count = int(desc.shape[0])
        self.total_keys = int(total_keys)
        self.max_segment_keys = int(max_segment_keys)
        self.d_desc = torch.from_numpy(desc.view(_np.uint8).copy()).to(device)

    def workspace_bytes(self):
        return sort_segmented_workspace_bytes(self.count, self.total_keys, self.max_segment_keys)

    def run(self, workspace=None, stream=None, tuning=None, flags=FS_FLAG_NONE):
        """One fs_sort_segmented call (fs_sort_segmented_tuned when `tuning`
        is given); `flags` is the key order of every segment (order_flags).
        Returns the workspace."""
        ws = workspace or Workspace(self.d_desc.device)
        buf = ws.get(self.workspace_bytes())
        size = ctypes.c_size_t(buf.numel())
        s = stream if stream is not None else torch.cuda.current_stream(self.d_desc.device)
        if tuning is None:
            st = lib().fs_sort_segmented(_ptr(self.d_desc), self.count, self.total_keys,
                                         self.max_segment_keys, flags, _ptr(buf), ctypes.byref(size),
                                         ctypes.c_void_p(s.cuda_stream))
        else:
            st = lib().fs_sort_segmented_tuned(_ptr(self.d_desc), self.count, self.total_keys,
                                               self.max_segment_keys, flags, ctypes.byref(tuning), _ptr(buf),
                                               ctypes.byref(size), ctypes.c_void_p(s.cuda_stream))
        if st != FS_OK:
            raise FsError(st, "fs_sort_segmented")
        return ws


class CapturedSort:
    """A hipGraph of one sort call, replayed with `replay()`.

    The library issues no memset and allocates nothing inside a call, so its
    whole launch sequence (fills, histograms, plan, passes) can be captured.
    The graph keeps the buffer addresses it was captured with; for a
    segmented sort the descriptors are read from device memory at run time,
    so new data in the same buffers, or rewritten descriptors, are sorted by
    a replay.
    """

    def __init__(self, fn, device="cuda"):
        self.graph = torch.cuda.CUDAGraph()
        torch.cuda.synchronize(device)
        side = torch.cuda.Stream(device)  # default priority
        side.wait_stream(torch.cuda.current_stream(device))
        with torch.cuda.stream(side):
            fn()  # warm-up outside capture (first-touch, occupancy queries)
        torch.cuda.current_stream(device).wait_stream(side)
        torch.cuda.synchronize(device)
        with torch.cuda.graph(self.graph):
            fn()

    def replay(self):
        self.graph.replay()


def sort_segmented(segments, workspace=None, tuning=None, key_type=None, descending=False):
    """Sort every (keys_in, keys_out, vals_in, vals_out) segment independently
    in one call; returns the workspace (its error word is 0 on success).
    One key order holds for every segment: `key_type` None follows the key
    dtypes, which must then agree on it (see order_flags)."""
    flags = {order_flags(seg[0], key_type, descending) for seg in segments} or {FS_FLAG_NONE}
    if len(flags) != 1:
        raise ValueError("segments of one call share one key order; pass key_type explicitly")
    return SegmentBatch(segments).run(workspace, tuning=tuning, flags=flags.pop())


# ------------------------------------------------------- batch stream sorting
# 16-bit keys: the 2^16-bin histogram is the whole multiset, so a stream of
# batches is sorted by accumulating their histograms and expanding the sum.

def _u16(t, what):
    if t.dtype not in (torch.uint16, torch.int16, torch.float16, torch.bfloat16):
        raise TypeError(f"{what} must hold 16-bit keys, not {t.dtype}")


def new_hist16(device="cuda"):
    """A zeroed resident 2^16-bin histogram (int64 tensor holding uint64 counts)."""
    return torch.zeros(65536, dtype=torch.int64, device=device)


def hist16_accumulate(keys, hist, workspace=None, key_type=None, descending=False):
    """hist[v] += number of keys of rank v in the key order (unsigned
    ascending: the keys equal to v); keys: 1-D 16-bit device tensor."""
    _check_dev(keys, hist)
    _u16(keys, "keys")
    if hist.dtype != torch.int64 or hist.numel() != 65536:
        raise ValueError("hist must be an int64 tensor of 65536 counts")
    n = keys.numel()
    L = lib()
    size = ctypes.c_size_t(0)
    flags = order_flags(keys, key_type, descending)
    st = L.fs_hist16_accumulate(None, n, flags, None, None, ctypes.byref(size), None)
    if st != FS_OK:
        raise FsError(st, "fs_hist16_accumulate (workspace query)")
    ws = workspace or Workspace(keys.device)
    buf = ws.get(size.value)
    size = ctypes.c_size_t(buf.numel())
    st = L.fs_hist16_accumulate(_ptr(keys), n, flags, _ptr(hist), _ptr(buf), ctypes.byref(size), _stream(keys))
    if st != FS_OK:
        raise FsError(st, "fs_hist16_accumulate")
    return hist


def hist16_prefix(hist, prefix=None):
    """Exclusive prefix of a 2^16-bin histogram: int64 tensor of 65537 (last = total)."""
    _check_dev(hist)
    prefix = torch.empty(65537, dtype=torch.int64, device=hist.device) if prefix is None else prefix
    _check_dev(prefix)
    st = lib().fs_hist16_prefix(_ptr(hist), _ptr(prefix), _stream(hist))
    if st != FS_OK:
        raise FsError(st, "fs_hist16_prefix")
    return prefix


def expand16(prefix, first, count, out=None, key_type="unsigned", descending=False):
    """Sorted positions [first, first + count) of the multiset `prefix`
    describes (key_type/descending: the order its histogram was built in)."""
    _check_dev(prefix)
    out = torch.empty(int(count), dtype=torch.uint16, device=prefix.device) if out is None else out
    _check_dev(out)
    _u16(out, "out")
    if out.numel() < count:
        raise ValueError("out is shorter than count")
    flags = order_flags(out, key_type, descending)
    st = lib().fs_expand16(_ptr(prefix), int(first), int(count), flags, _ptr(out), _stream(prefix))
    if st != FS_OK:
        raise FsError(st, "fs_expand16")
    return out


def sort16_host_workspace_bytes(batch_keys):
    size = ctypes.c_size_t(0)
    st = lib().fs_sort16_host(None, None, 0, int(batch_keys), 0, None, ctypes.byref(size), None, None)
    if st != FS_OK:
        raise FsError(st, "fs_sort16_host (workspace query)")
    return size.value


def sort16_host(keys, out=None, batch_keys=1 << 26, workspace=None, copy_stream=None, device="cuda",
                key_type=None, descending=False):
    """Sort 16-bit keys held in HOST memory (a CPU tensor, ideally pinned),
    streaming them through the device in batches of `batch_keys`.  `out` may
    be `keys` itself (in-place).  Blocks until `out` holds the result."""
    for t in (keys,) + ((out,) if out is not None else ()):
        if t.is_cuda or not t.is_contiguous():
            raise ValueError("sort16_host takes contiguous host tensors")
    _u16(keys, "keys")
    out = torch.empty(keys.shape, dtype=keys.dtype, pin_memory=keys.is_pinned()) if out is None else out
    _u16(out, "out")
    if out.numel() != keys.numel():
        raise ValueError("keys and out differ in length")
    dev = torch.device(device)
    ws = workspace or Workspace(dev)
    buf = ws.get(sort16_host_workspace_bytes(batch_keys))
    size = ctypes.c_size_t(buf.numel())
    xs = copy_stream if copy_stream is not None else torch.cuda.Stream(dev)
    cs = torch.cuda.current_stream(dev)
    st = lib().fs_sort16_host(_ptr(keys), _ptr(out), keys.numel(), int(batch_keys),
                              order_flags(keys, key_type, descending), _ptr(buf), ctypes.byref(size),
                              ctypes.c_void_p(xs.cuda_stream), ctypes.c_void_p(cs.cuda_stream))
    if st != FS_OK:
        raise FsError(st, "fs_sort16_host")
    return out


def sort_host(keys, out=None, batch_keys=1 << 26, device_keys=1 << 30, workspace=None, copy_stream=None,
              device="cuda", key_type=None, descending=False):
    """Sort 32- or 64-bit keys held in HOST memory (a CPU tensor, ideally
    pinned) that need not fit on the device: an MSD spill through ranges of
    at most `device_keys` keys.  Blocks until `out` holds the result."""
    if keys.is_cuda or not keys.is_contiguous():
        raise ValueError("sort_host takes a contiguous host tensor")
    bits = _key_bits(keys)
    if bits not in (32, 64):
        raise TypeError("sort_host takes 32- or 64-bit keys (16-bit keys: sort16_host)")
    out = torch.empty(keys.shape, dtype=keys.dtype, pin_memory=keys.is_pinned()) if out is None else out
    if out.is_cuda or out.numel() != keys.numel() or out.dtype != keys.dtype:
        raise ValueError("out must be a host tensor like keys")
    dev = torch.device(device)
    L = lib()
    size = ctypes.c_size_t(0)
    flags = order_flags(keys, key_type, descending)
    st = L.fs_sort_host(None, None, 0, bits, int(batch_keys), int(device_keys), flags, None, ctypes.byref(size),
                        None, None)
    if st != FS_OK:
        raise FsError(st, "fs_sort_host (workspace query)")
    ws = workspace or Workspace(dev)
    buf = ws.get(size.value)
    size = ctypes.c_size_t(buf.numel())
    xs = copy_stream if copy_stream is not None else torch.cuda.Stream(dev)
    cs = torch.cuda.current_stream(dev)
    st = L.fs_sort_host(_ptr(keys), _ptr(out), keys.numel(), bits, int(batch_keys), int(device_keys), flags,
                        _ptr(buf), ctypes.byref(size), ctypes.c_void_p(xs.cuda_stream),
                        ctypes.c_void_p(cs.cuda_stream))
    if st != FS_OK:
        raise FsError(st, "fs_sort_host")
    return out
