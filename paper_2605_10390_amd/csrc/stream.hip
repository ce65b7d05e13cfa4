// Batch stream sorting of 16-bit keys (include/fs_sort.h, fs_hist16_* /
// fs_expand16 / fs_sort16_host).  Host code only.
//
// For 16-bit keys the 2^16-bin histogram is the whole multiset, so a stream
// of batches is sorted by adding each batch's compressed histogram into one
// resident 64-bit histogram (the batch cache of Section III-C) and writing
// the sorted keys from its prefix at the end (Algorithm 5 with no trailing
// bits).  Batches never need to be resident together: fs_sort16_host feeds
// host memory through two device staging slots, copying batch b + 1 in on
// one stream while batch b is counted on another, then writes the output
// out through the same slots in chunks.
#include "fs_sort.h"
#include "fs_device.hpp"
#include "fs_internal.hpp"

#include <algorithm>

namespace fs {
namespace {

size_t align256(size_t x) { return (x + 255) / 256 * 256; }
bool aligned(const void* p, uint64_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }
constexpr uint64_t kMaxStreamKeys = 1ull << 36;
constexpr size_t kHistBytes = 8ull * 65536;
constexpr size_t kPrefixBytes = 8ull * 65537;

// workgroups of the compressed histogram of a batch of n keys: one per CU
// at most, none with fewer than 2^16 keys
uint32_t hist_groups(uint64_t n) {
    const uint64_t g = std::max<uint64_t>((n + 65535) / 65536, 1);
    return (uint32_t)std::min<uint64_t>(g, (uint64_t)device_cu_count());
}

size_t accumulate_bytes(uint64_t n) {
    return align256(4ull * hist_groups(n) * kHist16Words) + align256(4ull * 2 * kHist16Words);
}

// d_hist += histogram of keys[0, n) (n > 0), with `ws` of accumulate_bytes(n)
hipError_t enqueue_accumulate(const uint16_t* keys, uint64_t n, uint64_t* d_hist, char* ws, hipStream_t s) {
    const uint32_t groups = hist_groups(n);
    uint32_t* part = reinterpret_cast<uint32_t*>(ws);
    uint32_t* wrap = reinterpret_cast<uint32_t*>(ws + align256(4ull * groups * kHist16Words));
    hipError_t e = launch_fill_u32(wrap, 2ull * kHist16Words, 0, s);
    if (e == hipSuccess) e = launch_hist16c(keys, n, groups, part, wrap, wrap + kHist16Words, s);
    if (e == hipSuccess) e = launch_merge16(part, groups, wrap, wrap + kHist16Words, d_hist, s, true);
    return e;
}

// Events of the two staging slots of fs_sort16_host, destroyed on scope exit.
struct SlotEvents {
    hipEvent_t filled[2] = {nullptr, nullptr};   // a batch or chunk is in the slot
    hipEvent_t emptied[2] = {nullptr, nullptr};  // the slot may be overwritten
    bool ok = true;
    SlotEvents() {
        for (int i = 0; i < 2; ++i) {
            ok = ok && hipEventCreateWithFlags(&filled[i], hipEventDisableTiming) == hipSuccess;
            ok = ok && hipEventCreateWithFlags(&emptied[i], hipEventDisableTiming) == hipSuccess;
        }
    }
    ~SlotEvents() {
        for (int i = 0; i < 2; ++i) {
            if (filled[i]) (void)hipEventDestroy(filled[i]);
            if (emptied[i]) (void)hipEventDestroy(emptied[i]);
        }
    }
};

}  // namespace
}  // namespace fs

extern "C" {

fs_status fs_hist16_accumulate(const void* keys, uint64_t n, uint64_t* d_hist, void* workspace,
                               size_t* workspace_bytes, void* stream) {
    using namespace fs;
    if (!workspace_bytes || n > kMaxStreamKeys) return FS_ERR_INVALID_ARG;
    const size_t need = accumulate_bytes(n);
    if (!workspace) {
        *workspace_bytes = need;
        return FS_OK;
    }
    if (*workspace_bytes < need) return FS_ERR_WORKSPACE_TOO_SMALL;
    if (!d_hist || (n && !keys) || !aligned(workspace, 256) || !aligned(d_hist, 8) ||
        (keys && !aligned(keys, 2)))
        return FS_ERR_INVALID_ARG;
    if (n == 0) return FS_OK;
    const uintptr_t k = reinterpret_cast<uintptr_t>(keys), h = reinterpret_cast<uintptr_t>(d_hist),
                    w = reinterpret_cast<uintptr_t>(workspace);
    if ((k < h + kHistBytes && h < k + 2 * n) || (w < h + kHistBytes && h < w + need))
        return FS_ERR_INVALID_ARG;
    if (enqueue_accumulate(static_cast<const uint16_t*>(keys), n, d_hist, static_cast<char*>(workspace),
                           static_cast<hipStream_t>(stream)) != hipSuccess)
        return FS_ERR_DEVICE;
    return FS_OK;
}

fs_status fs_hist16_prefix(const uint64_t* d_hist, uint64_t* d_prefix, void* stream) {
    using namespace fs;
    if (!d_hist || !d_prefix || !aligned(d_hist, 8) || !aligned(d_prefix, 8)) return FS_ERR_INVALID_ARG;
    const uintptr_t h = reinterpret_cast<uintptr_t>(d_hist), p = reinterpret_cast<uintptr_t>(d_prefix);
    if (h < p + kPrefixBytes && p < h + kHistBytes) return FS_ERR_INVALID_ARG;
    if (launch_scan16(d_hist, d_prefix, static_cast<hipStream_t>(stream)) != hipSuccess) return FS_ERR_DEVICE;
    return FS_OK;
}

fs_status fs_expand16(const uint64_t* d_prefix, uint64_t first, uint64_t count, void* keys_out, void* stream) {
    using namespace fs;
    if (count > kMaxStreamKeys || first > kMaxStreamKeys) return FS_ERR_INVALID_ARG;
    if (count == 0) return FS_OK;
    if (!d_prefix || !keys_out || !aligned(d_prefix, 8) || !aligned(keys_out, 2)) return FS_ERR_INVALID_ARG;
    const uintptr_t p = reinterpret_cast<uintptr_t>(d_prefix), o = reinterpret_cast<uintptr_t>(keys_out);
    if (p < o + 2 * count && o < p + kPrefixBytes) return FS_ERR_INVALID_ARG;
    if (launch_expand16(d_prefix, static_cast<uint16_t*>(keys_out), first, count,
                        static_cast<hipStream_t>(stream)) != hipSuccess)
        return FS_ERR_DEVICE;
    return FS_OK;
}

fs_status fs_sort16_host(const void* h_keys_in, void* h_keys_out, uint64_t n, uint64_t batch_keys,
                         void* workspace, size_t* workspace_bytes, void* copy_stream, void* compute_stream) {
    using namespace fs;
    if (!workspace_bytes || n > kMaxStreamKeys || batch_keys == 0 || batch_keys > kMaxStreamKeys)
        return FS_ERR_INVALID_ARG;
    const uint64_t batch = (batch_keys + 7) / 8 * 8;  // slots start 16-byte aligned
    const size_t slot_bytes = align256(2 * batch);
    const size_t acc = accumulate_bytes(batch);
    const size_t need = align256(kHistBytes) + align256(kPrefixBytes) + acc + 2 * slot_bytes;
    if (!workspace) {
        *workspace_bytes = need;
        return FS_OK;
    }
    if (*workspace_bytes < need) return FS_ERR_WORKSPACE_TOO_SMALL;
    if ((n && (!h_keys_in || !h_keys_out)) || !aligned(workspace, 256) || (h_keys_in && !aligned(h_keys_in, 2)) ||
        (h_keys_out && !aligned(h_keys_out, 2)))
        return FS_ERR_INVALID_ARG;
    if (h_keys_in != h_keys_out && n &&
        reinterpret_cast<uintptr_t>(h_keys_in) < reinterpret_cast<uintptr_t>(h_keys_out) + 2 * n &&
        reinterpret_cast<uintptr_t>(h_keys_out) < reinterpret_cast<uintptr_t>(h_keys_in) + 2 * n)
        return FS_ERR_INVALID_ARG;
    if (n == 0) return FS_OK;

    hipStream_t cs = static_cast<hipStream_t>(compute_stream);
    hipStream_t xs = static_cast<hipStream_t>(copy_stream);
    char* ws = static_cast<char*>(workspace);
    uint64_t* hist = reinterpret_cast<uint64_t*>(ws);
    uint64_t* prefix = reinterpret_cast<uint64_t*>(ws + align256(kHistBytes));
    char* acc_ws = ws + align256(kHistBytes) + align256(kPrefixBytes);
    uint16_t* slot[2] = {reinterpret_cast<uint16_t*>(acc_ws + acc),
                         reinterpret_cast<uint16_t*>(acc_ws + acc + slot_bytes)};
    const uint16_t* in = static_cast<const uint16_t*>(h_keys_in);
    uint16_t* out = static_cast<uint16_t*>(h_keys_out);

    SlotEvents ev;
    if (!ev.ok) return FS_ERR_DEVICE;
    bool ok = launch_fill_u32(reinterpret_cast<uint32_t*>(hist), 2 * 65536, 0, cs) == hipSuccess;
    // every batch: copy in on the copy stream, count on the compute stream
    const uint64_t batches = (n + batch - 1) / batch;
    for (uint64_t b = 0; ok && b < batches; ++b) {
        const int i = (int)(b & 1);
        const uint64_t off = b * batch, len = std::min(batch, n - off);
        if (b >= 2) ok = hipStreamWaitEvent(xs, ev.emptied[i], 0) == hipSuccess;
        ok = ok && hipMemcpyAsync(slot[i], in + off, 2 * len, hipMemcpyHostToDevice, xs) == hipSuccess;
        ok = ok && hipEventRecord(ev.filled[i], xs) == hipSuccess;
        ok = ok && hipStreamWaitEvent(cs, ev.filled[i], 0) == hipSuccess;
        ok = ok && enqueue_accumulate(slot[i], len, hist, acc_ws, cs) == hipSuccess;
        ok = ok && hipEventRecord(ev.emptied[i], cs) == hipSuccess;
    }
    ok = ok && launch_scan16(hist, prefix, cs) == hipSuccess;
    // every chunk: expand on the compute stream, copy out on the copy stream
    // (all copies in precede all copies out on that stream, so the output
    // may be the input buffer itself)
    for (uint64_t c = 0; ok && c < batches; ++c) {
        const int i = (int)(c & 1);
        const uint64_t off = c * batch, len = std::min(batch, n - off);
        if (c >= 2) ok = hipStreamWaitEvent(cs, ev.emptied[i], 0) == hipSuccess;
        ok = ok && launch_expand16(prefix, slot[i], off, len, cs) == hipSuccess;
        ok = ok && hipEventRecord(ev.filled[i], cs) == hipSuccess;
        ok = ok && hipStreamWaitEvent(xs, ev.filled[i], 0) == hipSuccess;
        ok = ok && hipMemcpyAsync(out + off, slot[i], 2 * len, hipMemcpyDeviceToHost, xs) == hipSuccess;
        ok = ok && hipEventRecord(ev.emptied[i], xs) == hipSuccess;
    }
    // the host output is complete only when both streams have drained
    const bool drained = hipStreamSynchronize(xs) == hipSuccess && hipStreamSynchronize(cs) == hipSuccess;
    return ok && drained ? FS_OK : FS_ERR_DEVICE;
}

}  // extern "C"
