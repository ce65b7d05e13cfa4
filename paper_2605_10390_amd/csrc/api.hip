// C ABI entry points (include/fs_sort.h): argument checks, workspace layout
// and the launch sequence of each call.  Host code only.
#include "fs_sort.h"
#include "fs_profile.h"
#include "fs_device.hpp"
#include "fs_internal.hpp"

#include <algorithm>
#include <mutex>

namespace fs {

int device_cu_count() {
    int dev = 0, c = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    if (hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || c <= 0)
        return 256;
    return c;
}

static size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }
static uint64_t ceil_div(uint64_t a, uint64_t b) { return (a + b - 1) / b; }
static int ceil_log2(uint64_t n) {
    int b = 0;
    while (b < 64 && (1ull << b) < n) ++b;
    return b;
}

SortLayout sort_layout(uint64_t n, int key_bytes, int val_bytes, int num_cus, bool clobber) {
    SortLayout L;
    L.key_bytes = key_bytes;
    L.val_bytes = val_bytes;
    L.digits = key_bytes;  // 8-bit digits
    L.expand16 = key_bytes == 2 && val_bytes == 0;

    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = align_up(off + std::max<size_t>(bytes, 1), 256);
        return o;
    };
    L.err = take(4);
    L.plan = take(4ull * kPlanWords);
    L.hist = take(8ull * 8 * kRadix);
    L.base = take(8ull * 8 * 2 * kRadix);
    if (L.expand16) {
        // compressed 2^16-bin histogram, its prefix, expansion
        L.hist_groups = (uint32_t)std::min<uint64_t>(std::max<uint64_t>(ceil_div(n, 1u << 16), 1), num_cus);
        L.part = take(4ull * L.hist_groups * kHist16Words);
        L.wrap = take(4ull * 2 * kHist16Words);
        L.h16 = take(8ull * 65536);
        L.p16 = take(8ull * 65537);
    } else {
        L.tile = (uint32_t)tiled_shape(key_bytes, val_bytes).tile();
        L.tiles = std::max<uint64_t>(ceil_div(n, L.tile), 1);
        L.tile_blocks = ceil_div(L.tiles, 65536 / L.tile);
        L.tile_supers = ceil_div(L.tile_blocks, kSuperBlock);
        L.hist_groups = (uint32_t)std::min<uint64_t>(L.tile_blocks, 4ull * num_cus);
        static const int per_cu[4][3] = {
            {tiled_scatter_per_cu(1, 0), tiled_scatter_per_cu(1, 4), tiled_scatter_per_cu(1, 8)},
            {0, tiled_scatter_per_cu(2, 4), tiled_scatter_per_cu(2, 8)},
            {tiled_scatter_per_cu(4, 0), tiled_scatter_per_cu(4, 4), tiled_scatter_per_cu(4, 8)},
            {tiled_scatter_per_cu(8, 0), tiled_scatter_per_cu(8, 4), tiled_scatter_per_cu(8, 8)}};
        const int ki = key_bytes == 1 ? 0 : key_bytes == 2 ? 1 : key_bytes == 4 ? 2 : 3, vi = val_bytes / 4;
        L.scatter_groups = (uint32_t)std::max(1, num_cus * std::max(1, per_cu[ki][vi]));
        L.part = take(4ull * L.hist_groups * L.digits * kRadix);
        L.th = take(2ull * kRadix * L.tiles);
        L.bsum = take(4ull * kRadix * L.tile_blocks);
        L.ssum = take(4ull * kRadix * L.tile_supers);
        L.sbase = take(8ull * kRadix * L.tile_supers);
        L.tile_tickets = take(4ull * kPlanSlots * kXcds * kTicketStride);
        // the sparse-trie plan is offered to wide keys from kTrieMinKeys on
        // (below that its extra launches cost more than passes it can save)
        L.trie = key_bytes >= 4 && n >= kTrieMinKeys;
        if (L.trie) {
            L.trie_list = take(8ull * kTrieLongMax);
            L.trie_count = take(4);
        }
        L.sink = take(16);
        L.pairs16 = key_bytes == 2;
        if (L.pairs16) {
            // first histogram: the compressed 2^16-bin histogram of the keys,
            // one workgroup per CU
            L.hist16_groups = (uint32_t)std::min<uint64_t>(L.tile_blocks, (uint64_t)num_cus);
            L.part16 = take(4ull * L.hist16_groups * kHist16Words);
            L.wrap = take(4ull * 2 * kHist16Words);
            L.h16 = take(8ull * 65536);
            L.p16 = take(8ull * 65537);
            // the keys' high bytes between the passes (one byte per key)
            L.narrow = take((size_t)n);
        }
        // the passes' second buffer: none with clobber (the input serves);
        // none for the keys of a 16-bit pair sort (its first pass writes
        // only their high bytes, which the second pass reads, and the
        // sorted keys are expanded from the histogram)
        L.clobber = clobber;
        if (!clobber && !L.pairs16) L.tmp_keys = take((size_t)n * key_bytes);
        if (!clobber && val_bytes) L.tmp_vals = take((size_t)n * val_bytes);
    }
    L.total = off;
    return L;
}

static bool overlaps(const void* a, uint64_t abytes, const void* b, uint64_t bbytes) {
    const uintptr_t x = reinterpret_cast<uintptr_t>(a), y = reinterpret_cast<uintptr_t>(b);
    return x < y + bbytes && y < x + abytes;
}

static bool aligned(const void* p, uint64_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }

constexpr uint64_t kMaxKeys = 1ull << 36;

#define FS_TRY(expr)                                   \
    do {                                               \
        if ((expr) != hipSuccess) return FS_ERR_DEVICE; \
    } while (0)

// enqueue `expr` (a launch) under the event recorder as kernel `kind`
#define FS_LAUNCH(kind, keys, expr) FS_TRY(timed((kind), (keys), s, [&]() { return (expr); }))

// Key order masks of order_map (fs_device.hpp) for the order flags; false
// for an unknown flag (FS_FLAG_CLOBBER_INPUT included: callers that accept
// it strip it first) or SIGNED together with FLOAT.
bool order_masks(unsigned flags, int key_bits, uint64_t* pos, uint64_t* neg) {
    const unsigned known = FS_FLAG_SIGNED | FS_FLAG_FLOAT | FS_FLAG_DESCENDING;
    if ((flags & ~known) || ((flags & FS_FLAG_SIGNED) && (flags & FS_FLAG_FLOAT))) return false;
    if ((flags & FS_FLAG_FLOAT) && key_bits == 8) return false;  // no 8-bit IEEE format
    const uint64_t all = key_bits == 64 ? ~0ull : (1ull << key_bits) - 1;
    const uint64_t sign = 1ull << (key_bits - 1);
    uint64_t p = 0, q = 0;
    if (flags & FS_FLAG_SIGNED) p = q = sign;
    if (flags & FS_FLAG_FLOAT) {
        p = sign;
        q = all;
    }
    if (flags & FS_FLAG_DESCENDING) {
        p ^= all;
        q ^= all;
    }
    *pos = p;
    *neg = q;
    return true;
}

static fs_status sort_impl(const void* keys_in, void* keys_out, const void* vals_in, void* vals_out,
                           uint64_t n, int key_bits, int val_bytes, unsigned flags, void* workspace,
                           size_t* workspace_bytes, hipStream_t s) {
    if (key_bits != 8 && key_bits != 16 && key_bits != 32 && key_bits != 64) return FS_ERR_INVALID_ARG;
    uint64_t opos = 0, oneg = 0;
    const bool clobber = (flags & FS_FLAG_CLOBBER_INPUT) != 0;
    if (!order_masks(flags & ~(unsigned)FS_FLAG_CLOBBER_INPUT, key_bits, &opos, &oneg)) return FS_ERR_INVALID_ARG;
    if (val_bytes != 0 && val_bytes != 4 && val_bytes != 8) return FS_ERR_INVALID_ARG;
    if (!workspace_bytes || n > kMaxKeys) return FS_ERR_INVALID_ARG;
    const int kb = key_bits / 8;
    const SortLayout L = sort_layout(n, kb, val_bytes, device_cu_count(), clobber);
    if (!workspace) {
        *workspace_bytes = L.total;
        return FS_OK;
    }
    if (n == 0) return FS_OK;
    if (!keys_in || !keys_out || (val_bytes && (!vals_in || !vals_out))) return FS_ERR_INVALID_ARG;
    if (!aligned(keys_in, kb) || !aligned(keys_out, kb) || !aligned(workspace, 256))
        return FS_ERR_INVALID_ARG;
    if (val_bytes && (!aligned(vals_in, val_bytes) || !aligned(vals_out, val_bytes)))
        return FS_ERR_INVALID_ARG;
    const uint64_t kbytes = n * kb, vbytes = n * val_bytes;
    if (overlaps(keys_in, kbytes, keys_out, kbytes)) return FS_ERR_INVALID_ARG;
    if (val_bytes) {
        if (overlaps(vals_in, vbytes, vals_out, vbytes) || overlaps(keys_in, kbytes, vals_in, vbytes) ||
            overlaps(keys_out, kbytes, vals_out, vbytes) || overlaps(keys_in, kbytes, vals_out, vbytes) ||
            overlaps(keys_out, kbytes, vals_in, vbytes))
            return FS_ERR_INVALID_ARG;
    }
    if (*workspace_bytes < L.total) return FS_ERR_WORKSPACE_TOO_SMALL;
    if (overlaps(workspace, L.total, keys_out, kbytes) || overlaps(workspace, L.total, keys_in, kbytes))
        return FS_ERR_INVALID_ARG;
    if (val_bytes && (overlaps(workspace, L.total, vals_in, vbytes) || overlaps(workspace, L.total, vals_out, vbytes)))
        return FS_ERR_INVALID_ARG;

    char* w = static_cast<char*>(workspace);
    uint32_t* err = reinterpret_cast<uint32_t*>(w + L.err);
    uint32_t* plan = reinterpret_cast<uint32_t*>(w + L.plan);
    uint64_t* hist = reinterpret_cast<uint64_t*>(w + L.hist);
    uint64_t* base = reinterpret_cast<uint64_t*>(w + L.base);
    uint32_t* part = reinterpret_cast<uint32_t*>(w + L.part);

    // every range that must start at zero, cleared by one launch
    ZeroRanges zero;
    zero.p[0] = err;
    zero.words[0] = 1;

    if (L.expand16) {
        // the whole key is one 16-bit digit: compressed histogram, prefix,
        // expansion (Algorithm 5 with no trailing bits)
        uint32_t* wrap = reinterpret_cast<uint32_t*>(w + L.wrap);
        uint64_t* h16 = reinterpret_cast<uint64_t*>(w + L.h16);
        uint64_t* p16 = reinterpret_cast<uint64_t*>(w + L.p16);
        zero.p[1] = wrap;
        zero.words[1] = 2ull * kHist16Words;
        FS_LAUNCH(FS_KERNEL_AUX, 0, launch_zero(zero, s));
        FS_LAUNCH(FS_KERNEL_HISTOGRAM, n, launch_hist16c(static_cast<const uint16_t*>(keys_in), n, L.hist_groups,
                                                         part, wrap, wrap + kHist16Words, s, (uint32_t)opos,
                                                         (uint32_t)oneg));
        FS_LAUNCH(FS_KERNEL_PLAN, 0, launch_merge16(part, L.hist_groups, wrap, wrap + kHist16Words, h16, s));
        FS_LAUNCH(FS_KERNEL_PLAN, 0, launch_scan16(h16, p16, s));
        FS_LAUNCH(FS_KERNEL_EXPAND, n, launch_expand16(p16, static_cast<uint16_t*>(keys_out), 0, n, s, (uint32_t)opos,
                                                         (uint32_t)oneg));
        return FS_OK;
    }

    TiledArgs a;
    a.in_k = keys_in;
    a.out_k = keys_out;
    // the passes' second buffer (finish_plan's kBufTmp): the input itself
    // with clobber, the output for the keys of a 16-bit pair sort
    a.tmp_k = L.clobber ? const_cast<void*>(keys_in) : L.pairs16 ? keys_out : static_cast<void*>(w + L.tmp_keys);
    a.in_v = vals_in;
    a.out_v = vals_out;
    a.tmp_v = !val_bytes ? nullptr : L.clobber ? const_cast<void*>(vals_in) : static_cast<void*>(w + L.tmp_vals);
    a.n = n;
    a.tiles = L.tiles;
    a.tile = L.tile;
    a.block_tiles = 65536 / L.tile;
    a.plan = plan;
    a.base = base;
    a.th = reinterpret_cast<uint32_t*>(w + L.th);
    a.bsum = reinterpret_cast<uint32_t*>(w + L.bsum);
    a.ssum = reinterpret_cast<uint32_t*>(w + L.ssum);
    a.sbase = reinterpret_cast<uint64_t*>(w + L.sbase);
    a.part = part;
    a.tickets = reinterpret_cast<uint32_t*>(w + L.tile_tickets);
    a.sink = w + L.sink;
    a.err = err;
    a.ord_pos = opos;
    a.ord_neg = oneg;
    zero.p[1] = a.tickets;
    zero.words[1] = (uint64_t)kPlanSlots * kXcds * kTicketStride;
    if (L.trie) {
        a.trie_list = reinterpret_cast<uint64_t*>(w + L.trie_list);
        a.trie_count = reinterpret_cast<uint32_t*>(w + L.trie_count);
        zero.p[2] = a.trie_count;
        zero.words[2] = 1;
    }
    if (L.pairs16) {
        zero.p[2] = reinterpret_cast<uint32_t*>(w + L.wrap);
        zero.words[2] = 2ull * kHist16Words;
    }
    FS_LAUNCH(FS_KERNEL_AUX, 0, launch_zero(zero, s));
    if (L.pairs16) {
        // 16-bit keys with payloads: the first histogram is the compressed
        // 2^16-bin histogram (plus digit-0 tile counts); the last pass moves
        // only payloads and the sorted keys are expanded from the histogram
        uint32_t* part16 = reinterpret_cast<uint32_t*>(w + L.part16);
        uint32_t* wrap = reinterpret_cast<uint32_t*>(w + L.wrap);
        uint64_t* h16 = reinterpret_cast<uint64_t*>(w + L.h16);
        uint64_t* p16 = reinterpret_cast<uint64_t*>(w + L.p16);
        FS_LAUNCH(FS_KERNEL_HISTOGRAM, n,
                  launch_tile_hist16(a, L.hist16_groups, part16, wrap, wrap + kHist16Words, s));
        FS_LAUNCH(FS_KERNEL_PLAN, 0, launch_merge16(part16, L.hist16_groups, wrap, wrap + kHist16Words, h16, s));
        FS_LAUNCH(FS_KERNEL_PLAN, 0, launch_plan_from16(h16, n, hist, base, plan, s, L.clobber));
        FS_LAUNCH(FS_KERNEL_PLAN, 0, launch_scan16(h16, p16, s));
        // pass 0 writes the payloads and, into the workspace, the high byte
        // of every mapped key; pass 1 (when it runs, the last) sorts the
        // payloads by those bytes, read as one-byte keys that need no
        // further mapping.  (With those bytes in the output key buffer
        // instead, 2^30 pairs with 8-byte payloads measured 6% slower.)
        a.narrow = reinterpret_cast<uint8_t*>(w + L.narrow);
        TiledArgs an = a;
        an.ord_pos = an.ord_neg = 0;
        FS_LAUNCH(FS_KERNEL_PLAN, 0, launch_tile_offsets(a, 0, s));
        FS_LAUNCH(FS_KERNEL_SCATTER, n, launch_tile_scatter(a, kb, val_bytes, 0, L.scatter_groups, s));
        FS_LAUNCH(FS_KERNEL_AUX, 0, launch_narrow_copy(a, s));
        FS_LAUNCH(FS_KERNEL_HISTOGRAM, n, launch_tile_hist(an, 1, 1, L.hist_groups, s, false));
        FS_LAUNCH(FS_KERNEL_PLAN, 0, launch_tile_offsets(an, 1, s));
        FS_LAUNCH(FS_KERNEL_SCATTER, n, launch_tile_scatter_narrow(an, val_bytes, 1, L.scatter_groups, s));
        FS_LAUNCH(FS_KERNEL_AUX, 0, launch_copy_if(plan, vals_in, vals_out, vbytes, s));
        FS_LAUNCH(FS_KERNEL_EXPAND, n, launch_expand16(p16, static_cast<uint16_t*>(keys_out), 0, n, s, (uint32_t)opos,
                                                         (uint32_t)oneg));
        return FS_OK;
    }
    // sparse keys (n far below 2^p): the plan may sort only a window of the
    // top ceil(log2 n) bits and leave the trailing bits to the fixup
    const int trie_bits = L.trie ? ceil_log2(n) : 0;
    FS_LAUNCH(FS_KERNEL_HISTOGRAM, n, launch_tile_hist(a, kb, 0, L.hist_groups, s, true));
    FS_LAUNCH(FS_KERNEL_PLAN, 0, launch_tile_plan(part, L.hist_groups, L.digits, n, hist, base, plan, s, L.clobber,
                                                  trie_bits));
    auto run_slot = [&](int j) -> fs_status {
        if (j > 0 || trie_bits) FS_LAUNCH(FS_KERNEL_HISTOGRAM, n, launch_tile_hist(a, kb, j, L.hist_groups, s, false));
        FS_LAUNCH(FS_KERNEL_PLAN, 0, launch_tile_offsets(a, j, s));
        FS_LAUNCH(FS_KERNEL_SCATTER, n, launch_tile_scatter(a, kb, val_bytes, j, L.scatter_groups, s));
        return FS_OK;
    };
    for (int j = 0; j < L.digits; ++j)
        if (run_slot(j) != FS_OK) return FS_ERR_DEVICE;
    if (trie_bits) {
        FS_LAUNCH(FS_KERNEL_AUX, n, launch_trie_fixup(a, kb, val_bytes, s));
        FS_LAUNCH(FS_KERNEL_AUX, 0, launch_trie_longruns(a, kb, val_bytes, s));
        for (int j = kPlanCondSlot; j < kPlanCondSlot + L.digits; ++j)
            if (run_slot(j) != FS_OK) return FS_ERR_DEVICE;
    }
    FS_LAUNCH(FS_KERNEL_AUX, 0, launch_copy_if(plan, keys_in, keys_out, kbytes, s));
    if (val_bytes) FS_LAUNCH(FS_KERNEL_AUX, 0, launch_copy_if(plan, vals_in, vals_out, vbytes, s));
    if (trie_bits) {
        FS_LAUNCH(FS_KERNEL_AUX, 0, launch_copy_if(plan, a.tmp_k, keys_out, kbytes, s, kPlanCopyTmp));
        if (val_bytes) FS_LAUNCH(FS_KERNEL_AUX, 0, launch_copy_if(plan, a.tmp_v, vals_out, vbytes, s, kPlanCopyTmp));
    }
    return FS_OK;
}

// ---------------------------------------------------------------------------
// Allocation-free sorts (fs_sort_keys_noalloc): the workspace is `scratch`,
// a file-scope device array of FS_NOALLOC_SCRATCH_BYTES that every GPU the
// library runs on holds until the process ends.  Host code never passes the
// array's name to a kernel (on the host it is only a stand-in symbol): each
// device's address comes from hipGetSymbolAddress, taken once per device
// with that device current, and only that address is handed on.
// ---------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[FS_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

// The current device's copy of `scratch` (looked up on first use).
static fs_status scratch_address(void** out) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return FS_ERR_DEVICE;
    if (dev < 0 || dev >= kMaxDevices) return FS_ERR_UNSUPPORTED;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return FS_ERR_DEVICE;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return FS_OK;
}

static fs_status sort_keys_noalloc_impl(const void* keys_in, void* keys_out, uint64_t n, int key_bits,
                                        unsigned flags, uint32_t* err_out, hipStream_t s) {
    size_t need = 0;
    fs_status st = sort_impl(nullptr, nullptr, nullptr, nullptr, n, key_bits, 0, flags, nullptr, &need, s);
    if (st != FS_OK) return st;
    if (need > (size_t)FS_NOALLOC_SCRATCH_BYTES) return FS_ERR_WORKSPACE_TOO_SMALL;
    void* ws = nullptr;
    st = scratch_address(&ws);
    if (st != FS_OK) return st;
    size_t have = FS_NOALLOC_SCRATCH_BYTES;
    {
        const ProfileSuspend quiet;  // no timing events: they would be created on demand
        st = sort_impl(keys_in, keys_out, nullptr, nullptr, n, key_bits, 0, flags, ws, &have, s);
    }
    if (st != FS_OK || !err_out) return st;
    // word 0 of the workspace is the call's error word (0 for n == 0: the
    // word is then copied as the last call left it, so clear it first)
    if (n == 0) FS_TRY(launch_fill_u32(static_cast<uint32_t*>(ws), 1, 0, s));
    FS_TRY(hipMemcpyAsync(err_out, ws, 4, hipMemcpyDeviceToDevice, s));
    return FS_OK;
}

// Keys of `words` 64-bit words (word 0 least significant), sorted least
// significant word first: each round gathers one word of every key through
// the current permutation (mapped into the requested order) and stably sorts
// (word, permutation entry) pairs with sort_impl; the last permutation then
// moves whole keys and payloads.  Stable rounds from the lowest word up
// order keys by the highest word first, ties by the lower words, then by
// input position.
constexpr int kMaxKeyWords = 64;

static fs_status sort_wide_impl(const void* keys_in, void* keys_out, const void* vals_in, void* vals_out,
                                uint64_t n, int words, int val_bytes, unsigned flags, void* workspace,
                                size_t* workspace_bytes, hipStream_t s) {
    if (words < 1 || words > kMaxKeyWords) return FS_ERR_INVALID_ARG;
    if (val_bytes != 0 && val_bytes != 4 && val_bytes != 8) return FS_ERR_INVALID_ARG;
    if (!workspace_bytes || n > kMaxKeys) return FS_ERR_INVALID_ARG;
    if (words == 1)  // one word is a 64-bit key (inputs left as they are)
        return sort_impl(keys_in, keys_out, vals_in, vals_out, n, 64, val_bytes,
                         flags & ~(unsigned)FS_FLAG_CLOBBER_INPUT, workspace, workspace_bytes, s);
    // order masks per word: the top word carries the sign; a float's other
    // words are complemented when it is negative
    // the inputs are only gathered from, so CLOBBER_INPUT changes nothing
    flags &= ~(unsigned)FS_FLAG_CLOBBER_INPUT;
    const unsigned known = FS_FLAG_SIGNED | FS_FLAG_FLOAT | FS_FLAG_DESCENDING;
    if ((flags & ~known) || ((flags & FS_FLAG_SIGNED) && (flags & FS_FLAG_FLOAT))) return FS_ERR_INVALID_ARG;
    const uint64_t sign = 1ull << 63;
    auto word_masks = [&](int w, uint64_t* pos, uint64_t* neg) {
        uint64_t p = 0, q = 0;
        if (w == words - 1 && (flags & FS_FLAG_SIGNED)) p = q = sign;
        if (flags & FS_FLAG_FLOAT) {
            p = w == words - 1 ? sign : 0;
            q = ~0ull;
        }
        if (flags & FS_FLAG_DESCENDING) {
            p = ~p;
            q = ~q;
        }
        *pos = p;
        *neg = q;
    };
    const int pb = n > 0xFFFFFFFFull ? 8 : 4;  // permutation entry width
    size_t inner = 0;
    {
        const fs_status st = sort_impl(nullptr, nullptr, nullptr, nullptr, n, 64, pb, 0, nullptr, &inner, s);
        if (st != FS_OK) return st;
    }
    // the inner sort's workspace comes first, so word 0 is its error word
    const size_t o_inner = 0;
    const size_t o_perm0 = align_up(inner, 256);
    const size_t o_perm1 = o_perm0 + align_up(std::max<uint64_t>(n, 1) * pb, 256);
    const size_t o_word0 = o_perm1 + align_up(std::max<uint64_t>(n, 1) * pb, 256);
    const size_t o_word1 = o_word0 + align_up(std::max<uint64_t>(n, 1) * 8, 256);
    const size_t need = o_word1 + align_up(std::max<uint64_t>(n, 1) * 8, 256);
    if (!workspace) {
        *workspace_bytes = need;
        return FS_OK;
    }
    if (n == 0) return FS_OK;
    if (*workspace_bytes < need) return FS_ERR_WORKSPACE_TOO_SMALL;
    if (!keys_in || !keys_out || (val_bytes && (!vals_in || !vals_out))) return FS_ERR_INVALID_ARG;
    if (!aligned(keys_in, 8) || !aligned(keys_out, 8) || !aligned(workspace, 256)) return FS_ERR_INVALID_ARG;
    if (val_bytes && (!aligned(vals_in, val_bytes) || !aligned(vals_out, val_bytes))) return FS_ERR_INVALID_ARG;
    const uint64_t kbytes = n * 8ull * (uint64_t)words, vbytes = n * (uint64_t)val_bytes;
    if (overlaps(keys_in, kbytes, keys_out, kbytes) || overlaps(workspace, need, keys_in, kbytes) ||
        overlaps(workspace, need, keys_out, kbytes))
        return FS_ERR_INVALID_ARG;
    if (val_bytes && (overlaps(vals_in, vbytes, vals_out, vbytes) || overlaps(keys_in, kbytes, vals_in, vbytes) ||
                      overlaps(keys_out, kbytes, vals_out, vbytes) || overlaps(keys_in, kbytes, vals_out, vbytes) ||
                      overlaps(keys_out, kbytes, vals_in, vbytes) || overlaps(workspace, need, vals_in, vbytes) ||
                      overlaps(workspace, need, vals_out, vbytes)))
        return FS_ERR_INVALID_ARG;

    char* w = static_cast<char*>(workspace);
    void* perm[2] = {w + o_perm0, w + o_perm1};
    uint64_t* word[2] = {reinterpret_cast<uint64_t*>(w + o_word0), reinterpret_cast<uint64_t*>(w + o_word1)};
    int cur = 0;
    for (int r = 0; r < words; ++r) {
        uint64_t pos, neg;
        word_masks(r, &pos, &neg);
        FS_TRY(launch_gather_word(keys_in, (uint32_t)words, (uint32_t)r, r == 0 ? nullptr : perm[cur], pb, word[0],
                                  n, pos, neg, s));
        if (r == 0) FS_TRY(launch_iota(perm[cur], pb, n, s));
        size_t ib = inner;
        const fs_status st = sort_impl(word[0], word[1], perm[cur], perm[1 - cur], n, 64, pb, 0, w + o_inner, &ib, s);
        if (st != FS_OK) return st;
        cur = 1 - cur;
    }
    FS_TRY(launch_gather_keys(keys_in, keys_out, (uint32_t)words, perm[cur], pb, n, s));
    if (val_bytes) FS_TRY(launch_gather_vals(vals_in, vals_out, val_bytes, perm[cur], pb, n, s));
    return FS_OK;
}

}  // namespace fs

extern "C" {

fs_status fs_sort_keys(const void* keys_in, void* keys_out, uint64_t n, int key_bits, unsigned flags,
                       void* workspace, size_t* workspace_bytes, void* stream) {
    return fs::sort_impl(keys_in, keys_out, nullptr, nullptr, n, key_bits, 0, flags, workspace,
                         workspace_bytes, static_cast<hipStream_t>(stream));
}

fs_status fs_sort_keys_noalloc(const void* keys_in, void* keys_out, uint64_t n, int key_bits, unsigned flags,
                               uint32_t* err_out, void* stream) {
    return fs::sort_keys_noalloc_impl(keys_in, keys_out, n, key_bits, flags, err_out,
                                      static_cast<hipStream_t>(stream));
}

fs_status fs_sort_pairs(const void* keys_in, void* keys_out, const void* vals_in, void* vals_out,
                        uint64_t n, int key_bits, int val_bytes, unsigned flags, void* workspace,
                        size_t* workspace_bytes, void* stream) {
    if (val_bytes != 4 && val_bytes != 8) return FS_ERR_INVALID_ARG;
    return fs::sort_impl(keys_in, keys_out, vals_in, vals_out, n, key_bits, val_bytes, flags, workspace,
                         workspace_bytes, static_cast<hipStream_t>(stream));
}

fs_status fs_sort_keys_wide(const void* keys_in, void* keys_out, uint64_t n, int key_words, unsigned flags,
                            void* workspace, size_t* workspace_bytes, void* stream) {
    return fs::sort_wide_impl(keys_in, keys_out, nullptr, nullptr, n, key_words, 0, flags, workspace,
                              workspace_bytes, static_cast<hipStream_t>(stream));
}

fs_status fs_sort_pairs_wide(const void* keys_in, void* keys_out, const void* vals_in, void* vals_out, uint64_t n,
                             int key_words, int val_bytes, unsigned flags, void* workspace, size_t* workspace_bytes,
                             void* stream) {
    if (val_bytes != 4 && val_bytes != 8) return FS_ERR_INVALID_ARG;
    return fs::sort_wide_impl(keys_in, keys_out, vals_in, vals_out, n, key_words, val_bytes, flags, workspace,
                              workspace_bytes, static_cast<hipStream_t>(stream));
}

fs_status fs_digit_histograms(const void* keys, uint64_t n, int key_bits, int digit_bits,
                              uint64_t* hist_out, void* workspace, size_t* workspace_bytes,
                              void* stream) {
    using namespace fs;
    if (key_bits != 16 && key_bits != 32 && key_bits != 64) return FS_ERR_INVALID_ARG;
    if (digit_bits != 8 && !(digit_bits == 16 && key_bits == 16)) return FS_ERR_INVALID_ARG;
    if (!workspace_bytes || n > kMaxKeys) return FS_ERR_INVALID_ARG;
    const int kb = key_bits / 8;
    const int cus = device_cu_count();
    uint32_t groups;
    size_t need;
    if (digit_bits == 16) {
        groups = (uint32_t)std::min<uint64_t>(std::max<uint64_t>(ceil_div(n, 1u << 16), 1), cus);
        need = align_up(4ull * groups * kHist16Words, 256) + 4ull * 2 * kHist16Words;
    } else {
        groups = (uint32_t)std::min<uint64_t>(std::max<uint64_t>(ceil_div(n, (uint64_t)kHist8Threads * 16), 1),
                                              2ull * cus);
        need = 4ull * groups * kb * kRadix;
    }
    need = align_up(need, 256);
    if (!workspace) {
        *workspace_bytes = need;
        return FS_OK;
    }
    if (*workspace_bytes < need) return FS_ERR_WORKSPACE_TOO_SMALL;
    if (!hist_out || (n && !keys) || !aligned(workspace, 256) || !aligned(hist_out, 8) ||
        (keys && !aligned(keys, kb)))
        return FS_ERR_INVALID_ARG;
    hipStream_t s = static_cast<hipStream_t>(stream);
    uint32_t* part = static_cast<uint32_t*>(workspace);
    if (digit_bits == 16) {
        uint32_t* wrap = reinterpret_cast<uint32_t*>(static_cast<char*>(workspace) +
                                                     align_up(4ull * groups * kHist16Words, 256));
        FS_TRY(launch_fill_u32(wrap, 2ull * kHist16Words, 0, s));
        if (n) FS_TRY(launch_hist16c(static_cast<const uint16_t*>(keys), n, groups, part, wrap, wrap + kHist16Words, s));
        else FS_TRY(launch_fill_u32(part, kHist16Words, 0, s));
        FS_TRY(launch_merge16(part, n ? groups : 1, wrap, wrap + kHist16Words, hist_out, s));
    } else {
        if (n) FS_TRY(launch_hist8(keys, n, kb, groups, part, s));
        else FS_TRY(launch_fill_u32(part, (uint64_t)kb * kRadix, 0, s));
        FS_TRY(launch_reduce8(part, n ? groups : 1, kb, hist_out, s));
    }
    return FS_OK;
}

namespace {
// built-in defaults (what the autotuner picked for a log-normal mix of
// 16- and 32-bit segments on MI355X): the LDS bin takes whatever fits,
// 16-bit keys-only segments from 16384 keys take the 16-bit-digit bin (split
// from 2^18 keys, two workgroups per CU), other segments up to 2^17 keys get
// one workgroup each, tiles of 4096 keys, three workgroups per CU in the
// large bin and two in the LDS bin
constexpr fs_seg_tuning kDefaultTuning = {{0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu}, 16384u, 1u << 18, 2u, 1u << 17, 16u, 256u, 3u, 2u};
std::mutex g_tuning_mu;
fs_seg_tuning g_tuning = kDefaultTuning;
}  // namespace

fs_status fs_segmented_default_tuning(fs_seg_tuning* out) {
    if (!out) return FS_ERR_INVALID_ARG;
    *out = kDefaultTuning;
    return FS_OK;
}

fs_status fs_set_segmented_tuning(const fs_seg_tuning* tuning) {
    const fs_seg_tuning t = tuning ? *tuning : kDefaultTuning;
    if (!fs::seg_tuning_valid(t)) return FS_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(g_tuning_mu);
    g_tuning = t;
    return FS_OK;
}

fs_status fs_get_segmented_tuning(fs_seg_tuning* out) {
    if (!out) return FS_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(g_tuning_mu);
    *out = g_tuning;
    return FS_OK;
}

fs_status fs_sort_segmented(const fs_segment* d_segments, uint32_t num_segments, uint64_t total_keys,
                            uint64_t max_segment_keys, unsigned flags, void* workspace,
                            size_t* workspace_bytes, void* stream) {
    return fs_sort_segmented_tuned(d_segments, num_segments, total_keys, max_segment_keys, flags, nullptr,
                                   workspace, workspace_bytes, stream);
}

fs_status fs_sort_segmented_tuned(const fs_segment* d_segments, uint32_t num_segments, uint64_t total_keys,
                                  uint64_t max_segment_keys, unsigned flags, const fs_seg_tuning* tuning,
                                  void* workspace, size_t* workspace_bytes, void* stream) {
    using namespace fs;
    if (!workspace_bytes) return FS_ERR_INVALID_ARG;
    // CLOBBER_INPUT is accepted and changes nothing (segments have their
    // own temporary pools)
    flags &= ~(unsigned)FS_FLAG_CLOBBER_INPUT;
    uint64_t opos[3], oneg[3];  // key order masks per width (16, 32, 64 bits)
    for (int w = 0; w < 3; ++w)
        if (!order_masks(flags, 16 << w, &opos[w], &oneg[w])) return FS_ERR_INVALID_ARG;
    fs_seg_tuning tune;
    if (tuning) {
        tune = *tuning;
    } else {
        std::lock_guard<std::mutex> lk(g_tuning_mu);
        tune = g_tuning;
    }
    if (!seg_tuning_valid(tune)) return FS_ERR_INVALID_ARG;
    if (max_segment_keys > kSegMaxKeys) return FS_ERR_UNSUPPORTED;
    if (total_keys > kMaxKeys) return FS_ERR_INVALID_ARG;
    const uint32_t nseg = num_segments;
    const uint32_t max_tiles = seg_max_tiles(total_keys, nseg);
    const uint64_t nl_max = std::min<uint64_t>(nseg, total_keys / (kSegMinSmallMax + 1) + 1);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = align_up(off + std::max<size_t>(bytes, 1), 256);
        return o;
    };
    const size_t o_err = take(4 * (1 + 256));
    const size_t o_small = take(4ull * nseg);
    const size_t o_wave = take(4ull * nseg);
    const size_t o_expand = take(4ull * nseg);
    const uint64_t nx_max = std::min<uint64_t>(nseg, total_keys / kX16MinSplit);
    const size_t o_x16p = take(4ull * (nx_max + 1));
    const size_t o_x16h = take(4ull * 65536 * nx_max);
    const size_t o_large = take(4ull * 9 * nseg);
    const size_t o_wg = take(4ull * 9 * nseg);
    const size_t o_tp = take(4ull * (nseg + 1));
    const size_t o_ep = take(8ull * (nseg + 1));
    const size_t o_ts = take(4ull * max_tiles);
    const size_t o_hist = take(4ull * nl_max * 8 * kRadix);
    const size_t o_plan = take(4ull * nl_max * 9);
    const size_t o_state = take(4ull * max_tiles * kRadix);
    const size_t o_tdesc = take(sizeof(SegTileDesc) * (size_t)max_tiles);
    const size_t o_tk = take(8ull * total_keys);
    const size_t o_tv = take(8ull * total_keys);
    const size_t need = off;
    if (!workspace) {
        *workspace_bytes = need;
        return FS_OK;
    }
    if (nseg == 0) return FS_OK;
    if (!d_segments || !aligned(workspace, 256) || !aligned(d_segments, 8)) return FS_ERR_INVALID_ARG;
    if (*workspace_bytes < need) return FS_ERR_WORKSPACE_TOO_SMALL;
    hipStream_t s = static_cast<hipStream_t>(stream);
    char* w = static_cast<char*>(workspace);
    SegCtx x;
    x.ord = flags != FS_FLAG_NONE;
    for (int w = 0; w < 3; ++w) {
        x.ord_pos[w] = opos[w];
        x.ord_neg[w] = oneg[w];
    }
    x.segs = d_segments;
    x.nseg = nseg;
    x.max_seg = max_segment_keys;
    x.total_keys = total_keys;
    x.max_tiles = max_tiles;
    x.err = reinterpret_cast<uint32_t*>(w + o_err);
    x.ctr = x.err + 1;
    x.small_list = reinterpret_cast<uint32_t*>(w + o_small);
    x.wave_list = reinterpret_cast<uint32_t*>(w + o_wave);
    x.expand_list = reinterpret_cast<uint32_t*>(w + o_expand);
    x.x16_parts = reinterpret_cast<uint32_t*>(w + o_x16p);
    x.x16_hist = reinterpret_cast<uint32_t*>(w + o_x16h);
    x.large_list = reinterpret_cast<uint32_t*>(w + o_large);
    x.wg_list = reinterpret_cast<uint32_t*>(w + o_wg);
    x.tile_prefix = reinterpret_cast<uint32_t*>(w + o_tp);
    x.elem_prefix = reinterpret_cast<uint64_t*>(w + o_ep);
    x.tile_seg = reinterpret_cast<uint32_t*>(w + o_ts);
    x.hist = reinterpret_cast<uint32_t*>(w + o_hist);
    x.plan = reinterpret_cast<uint32_t*>(w + o_plan);
    x.state = reinterpret_cast<uint32_t*>(w + o_state);
    x.tdesc = reinterpret_cast<SegTileDesc*>(w + o_tdesc);
    x.tmp_k = w + o_tk;
    x.tmp_v = w + o_tv;
    ZeroRanges zero;
    zero.p[0] = x.err;
    zero.words[0] = 1 + 256;
    zero.p[1] = x.state;
    zero.words[1] = (uint64_t)max_tiles * kRadix;
    FS_LAUNCH(FS_KERNEL_AUX, 0, launch_zero(zero, s));
    FS_LAUNCH(FS_KERNEL_SEGMENTED, total_keys, launch_segmented(x, tune, s));
    return FS_OK;
}

const char* fs_status_string(fs_status s) {
    switch (s) {
    case FS_OK: return "FS_OK";
    case FS_ERR_INVALID_ARG: return "FS_ERR_INVALID_ARG";
    case FS_ERR_UNSUPPORTED: return "FS_ERR_UNSUPPORTED";
    case FS_ERR_WORKSPACE_TOO_SMALL: return "FS_ERR_WORKSPACE_TOO_SMALL";
    case FS_ERR_DEVICE: return "FS_ERR_DEVICE";
    default: return "FS_ERR_UNKNOWN";
    }
}

}  // extern "C"
