"""The C-ABI library loads and exports every symbol include/fs_sort.h
declares (no GPU needed: no compute call is made)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", h) for h in sorted(os.listdir(os.path.join(ROOT, "include")))
           if h.endswith(".h")]
LIB = os.path.join(ROOT, "paper_2605_10390_amd", "libfsort.so")


def declared_symbols():
    text = "".join(open(h).read() for h in HEADERS)
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fs_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_boundary():
    syms = declared_symbols()
    for s in ("fs_sort_keys", "fs_sort_pairs", "fs_sort_segmented", "fs_digit_histograms",
              "fs_status_string", "fs_profile_enable", "fs_profile_read"):
        assert s in syms


@pytest.mark.skipif(not os.path.exists(LIB), reason="libfsort.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    for s in declared_symbols():
        assert hasattr(lib, s), f"{s} not exported"
    lib.fs_status_string.restype = ctypes.c_char_p
    assert lib.fs_status_string(0) == b"FS_OK"
    assert lib.fs_status_string(3) == b"FS_ERR_WORKSPACE_TOO_SMALL"


@pytest.mark.skipif(not os.path.exists(LIB), reason="libfsort.so not built")
def test_argument_errors_need_no_gpu():
    """Invalid widths are rejected before any device call."""
    lib = ctypes.CDLL(LIB)
    size = ctypes.c_size_t(0)
    lib.fs_sort_keys.restype = ctypes.c_int
    lib.fs_sort_keys.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int,
                                 ctypes.c_uint, ctypes.c_void_p,
                                 ctypes.POINTER(ctypes.c_size_t), ctypes.c_void_p]
    assert lib.fs_sort_keys(None, None, 10, 24, 0, None, ctypes.byref(size), None) == 1
    # SIGNED with FLOAT, and an unknown flag bit, are rejected; valid flags are not
    assert lib.fs_sort_keys(None, None, 10, 16, 6, None, ctypes.byref(size), None) == 1
    assert lib.fs_sort_keys(None, None, 10, 16, 16, None, ctypes.byref(size), None) == 1
    for flags in (1, 2, 4, 8, 9, 10, 12, 13):
        assert lib.fs_sort_keys(None, None, 10, 32, flags, None, ctypes.byref(size), None) == 0
    # 8-bit keys take every order but FLOAT
    for flags in (0, 1, 2, 8, 11):
        assert lib.fs_sort_keys(None, None, 10, 8, flags, None, ctypes.byref(size), None) == 0
    assert lib.fs_sort_keys(None, None, 10, 8, 4, None, ctypes.byref(size), None) == 1


def _header_flags():
    text = open(os.path.join(ROOT, "include", "fs_sort.h")).read()
    return {m.group(1): int(m.group(2)) for m in re.finditer(r"\b(FS_FLAG_[A-Z_]+)\s*=\s*(\d+)", text)}


def test_flag_values_are_pinned():
    """The boundary's flag values: CLOBBER_INPUT is bit 0 (as the boundary
    was first stated), the key orders bits 1-3; the binding agrees."""
    import paper_2605_10390_amd as fs
    want = {"FS_FLAG_NONE": 0, "FS_FLAG_CLOBBER_INPUT": 1, "FS_FLAG_SIGNED": 2, "FS_FLAG_FLOAT": 4,
            "FS_FLAG_DESCENDING": 8}
    assert _header_flags() == want
    for name, v in want.items():
        assert getattr(fs, name) == v, name


@pytest.mark.skipif(not os.path.exists(LIB), reason="libfsort.so not built")
def test_clobber_drops_the_temporary_copy():
    """With FS_FLAG_CLOBBER_INPUT the workspace query shrinks by the
    temporary key and payload arrays, n * (key bytes + payload bytes), up to
    256-byte alignment; 16-bit pair sorts never hold a key copy; 16-bit
    keys-only sorts hold none either way."""
    lib = ctypes.CDLL(LIB)
    vp, u64, i32, ui = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int, ctypes.c_uint
    sz = ctypes.POINTER(ctypes.c_size_t)
    lib.fs_sort_keys.argtypes = [vp, vp, u64, i32, ui, vp, sz, vp]
    lib.fs_sort_pairs.argtypes = [vp, vp, vp, vp, u64, i32, i32, ui, vp, sz, vp]

    def query(bits, vb, flags, n):
        size = ctypes.c_size_t(0)
        if vb:
            st = lib.fs_sort_pairs(None, None, None, None, n, bits, vb, flags, None, ctypes.byref(size), None)
        else:
            st = lib.fs_sort_keys(None, None, n, bits, flags, None, ctypes.byref(size), None)
        assert st == 0
        return size.value

    n = (1 << 20) + 7
    for bits in (8, 16, 32, 64):
        for vb in (0, 4, 8):
            plain, clob = query(bits, vb, 0, n), query(bits, vb, 1, n)
            kb = bits // 8
            if bits == 16 and vb == 0:
                assert plain == clob
                continue
            tmp = (0 if bits == 16 else n * kb) + n * vb
            assert 0 <= (plain - clob) - tmp < 512, (bits, vb, plain, clob)
            # ordered sorts have the same layouts
            assert query(bits, vb, 1 | 8, n) == clob


@pytest.mark.skipif(not os.path.exists(LIB), reason="libfsort.so not built")
def test_extended_entry_points_check_arguments_without_a_gpu():
    """Workspace queries of the multi-word, stream and out-of-core sorts
    answer, and bad widths or flags are refused, before any device call."""
    lib = ctypes.CDLL(LIB)
    vp, u64, i32, ui = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int, ctypes.c_uint
    sz = ctypes.POINTER(ctypes.c_size_t)
    lib.fs_sort_keys_wide.argtypes = [vp, vp, u64, i32, ui, vp, sz, vp]
    lib.fs_sort_host.argtypes = [vp, vp, u64, i32, u64, u64, ui, vp, sz, vp, vp]
    lib.fs_sort16_host.argtypes = [vp, vp, u64, u64, ui, vp, sz, vp, vp]
    lib.fs_hist16_accumulate.argtypes = [vp, u64, ui, vp, vp, sz, vp]
    size = ctypes.c_size_t(0)
    for words in (0, 65):
        assert lib.fs_sort_keys_wide(None, None, 100, words, 0, None, ctypes.byref(size), None) == 1
    assert lib.fs_sort_keys_wide(None, None, 100, 3, 0, None, ctypes.byref(size), None) == 0
    assert size.value > 0
    assert lib.fs_sort_keys_wide(None, None, 100, 2, 6, None, ctypes.byref(size), None) == 1  # SIGNED|FLOAT
    assert lib.fs_sort_keys_wide(None, None, 100, 2, 1 | 2, None, ctypes.byref(size), None) == 0  # clobber accepted
    for bits in (8, 16, 24):
        assert lib.fs_sort_host(None, None, 10, bits, 64, 64, 0, None, ctypes.byref(size), None, None) == 1
    assert lib.fs_sort_host(None, None, 10, 32, 0, 64, 0, None, ctypes.byref(size), None, None) == 1
    assert lib.fs_sort_host(None, None, 10, 64, 64, 64, 2 | 8, None, ctypes.byref(size), None, None) == 0
    # the host-memory and stream calls take order flags only
    assert lib.fs_sort_host(None, None, 10, 64, 64, 64, 1, None, ctypes.byref(size), None, None) == 1
    assert lib.fs_sort16_host(None, None, 10, 64, 16, None, ctypes.byref(size), None, None) == 1
    assert lib.fs_sort16_host(None, None, 10, 64, 8, None, ctypes.byref(size), None, None) == 0
    assert lib.fs_hist16_accumulate(None, 10, 6, None, None, ctypes.byref(size), None) == 1
    assert lib.fs_hist16_accumulate(None, 10, 1, None, None, ctypes.byref(size), None) == 1
    assert lib.fs_hist16_accumulate(None, 10, 2, None, None, ctypes.byref(size), None) == 0


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    """Without the HIP library the binding raises; there is no CPU path."""
    import paper_2605_10390_amd as fs
    monkeypatch.setattr(fs, "_lib", None)
    monkeypatch.setattr(fs, "LIB_PATH", str(tmp_path / "libfsort.so"))
    with pytest.raises(RuntimeError, match="no CPU fallback"):
        fs.lib()
    with pytest.raises(RuntimeError, match="no CPU fallback"):
        fs.sort_keys_workspace_bytes(1000, 16)


@pytest.mark.skipif(not os.path.exists(LIB), reason="libfsort.so not built")
def test_noalloc_limits_need_no_gpu():
    """fs_sort_keys_noalloc refuses, before any device call, every (n, width,
    flags) whose fs_sort_keys workspace exceeds the static scratch array, and
    bad arguments as fs_sort_keys does."""
    lib = ctypes.CDLL(LIB)
    vp, sz = ctypes.c_void_p, ctypes.POINTER(ctypes.c_size_t)
    lib.fs_sort_keys.argtypes = [vp, vp, ctypes.c_uint64, ctypes.c_int, ctypes.c_uint, vp, sz, vp]
    lib.fs_sort_keys_noalloc.argtypes = [vp, vp, ctypes.c_uint64, ctypes.c_int, ctypes.c_uint, vp, vp]
    text = open(os.path.join(ROOT, "include", "fs_sort.h")).read()
    m = re.search(r"#define\s+FS_NOALLOC_SCRATCH_BYTES\s+\((\d+)ull\s*<<\s*(\d+)\)", text)
    cap = int(m.group(1)) << int(m.group(2))
    assert cap == 64 << 20

    def need(n, bits, flags):
        size = ctypes.c_size_t(0)
        assert lib.fs_sort_keys(None, None, n, bits, flags, None, ctypes.byref(size), None) == 0
        return size.value

    cases = [(1 << 30, 32, 1), (1 << 29, 64, 1), (1 << 24, 32, 0), (1 << 23, 64, 0)]
    for n, bits, flags in cases:
        assert need(n, bits, flags) > cap
        assert lib.fs_sort_keys_noalloc(None, None, n, bits, flags, None, None) == 3
    # sizes that fit are documented in the header: 16-bit keys at any n,
    # clobbered 32/64-bit keys to 2^28, others to 2^23 / 2^22
    for n, bits, flags in [(1 << 36, 16, 0), (1 << 36, 16, 1), (1 << 28, 32, 1), (1 << 28, 64, 1),
                           (1 << 23, 32, 0), (1 << 22, 64, 0)]:
        assert need(n, bits, flags) <= cap, (n, bits, flags)
    assert lib.fs_sort_keys_noalloc(None, None, 10, 24, 0, None, None) == 1
    assert lib.fs_sort_keys_noalloc(None, None, 10, 16, 6, None, None) == 1
