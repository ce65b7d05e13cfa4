// Batch stream sorting (include/fs_sort.h): fs_hist16_* / fs_expand16 /
// fs_sort16_host for 16-bit keys, fs_sort_host for 32- and 64-bit keys.
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
#include <cstring>
#include <vector>

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
hipError_t enqueue_accumulate(const uint16_t* keys, uint64_t n, uint64_t* d_hist, char* ws, hipStream_t s,
                              uint32_t opos = 0, uint32_t oneg = 0) {
    const uint32_t groups = hist_groups(n);
    uint32_t* part = reinterpret_cast<uint32_t*>(ws);
    uint32_t* wrap = reinterpret_cast<uint32_t*>(ws + align256(4ull * groups * kHist16Words));
    hipError_t e = launch_fill_u32(wrap, 2ull * kHist16Words, 0, s);
    if (e == hipSuccess) e = launch_hist16c(keys, n, groups, part, wrap, wrap + kHist16Words, s, opos, oneg);
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

fs_status fs_hist16_accumulate(const void* keys, uint64_t n, unsigned flags, uint64_t* d_hist, void* workspace,
                               size_t* workspace_bytes, void* stream) {
    using namespace fs;
    uint64_t opos, oneg;
    if (!workspace_bytes || n > kMaxStreamKeys || !order_masks(flags, 16, &opos, &oneg)) return FS_ERR_INVALID_ARG;
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
                           static_cast<hipStream_t>(stream), (uint32_t)opos, (uint32_t)oneg) != hipSuccess)
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

fs_status fs_expand16(const uint64_t* d_prefix, uint64_t first, uint64_t count, unsigned flags, void* keys_out,
                      void* stream) {
    using namespace fs;
    uint64_t opos, oneg;
    if (count > kMaxStreamKeys || first > kMaxStreamKeys || !order_masks(flags, 16, &opos, &oneg))
        return FS_ERR_INVALID_ARG;
    if (count == 0) return FS_OK;
    if (!d_prefix || !keys_out || !aligned(d_prefix, 8) || !aligned(keys_out, 2)) return FS_ERR_INVALID_ARG;
    const uintptr_t p = reinterpret_cast<uintptr_t>(d_prefix), o = reinterpret_cast<uintptr_t>(keys_out);
    if (p < o + 2 * count && o < p + kPrefixBytes) return FS_ERR_INVALID_ARG;
    if (launch_expand16(d_prefix, static_cast<uint16_t*>(keys_out), first, count, static_cast<hipStream_t>(stream),
                        (uint32_t)opos, (uint32_t)oneg) != hipSuccess)
        return FS_ERR_DEVICE;
    return FS_OK;
}

fs_status fs_sort16_host(const void* h_keys_in, void* h_keys_out, uint64_t n, uint64_t batch_keys, unsigned flags,
                         void* workspace, size_t* workspace_bytes, void* copy_stream, void* compute_stream) {
    using namespace fs;
    uint64_t opos, oneg;
    if (!workspace_bytes || n > kMaxStreamKeys || batch_keys == 0 || batch_keys > kMaxStreamKeys ||
        !order_masks(flags, 16, &opos, &oneg))
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
        ok = ok && enqueue_accumulate(slot[i], len, hist, acc_ws, cs, (uint32_t)opos, (uint32_t)oneg) == hipSuccess;
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
        ok = ok && launch_expand16(prefix, slot[i], off, len, cs, (uint32_t)opos, (uint32_t)oneg) == hipSuccess;
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

// ---------------------------------------------------------------------------
// Out-of-core sort of 32- and 64-bit keys (fs_sort_host): an MSD spill.  The
// 16 bits just below the highest bit on which keys differ split the key
// range into 2^16 ordered buckets; consecutive buckets are grouped into
// ranges that fit the device, and each range is gathered from the streamed
// input, sorted on the device and written to its place in the output.
// ---------------------------------------------------------------------------
namespace fs {
namespace {

constexpr int kHostThreads = 256;

// Every kernel here works on the order-mapped key (order_map with opos,
// oneg; both 0 for unsigned ascending) and moves the caller's bits.

// OR and AND of every key (the bits on which keys differ are OR ^ AND)
template <typename K>
__global__ __launch_bounds__(kHostThreads) void k_or_and(const K* __restrict__ keys, uint64_t n,
                                                         unsigned long long* acc, uint64_t opos, uint64_t oneg) {
    uint64_t o = 0, a = ~0ull;
    const uint64_t stride = (uint64_t)gridDim.x * kHostThreads;
    for (uint64_t i = (uint64_t)blockIdx.x * kHostThreads + threadIdx.x; i < n; i += stride) {
        const uint64_t t = order_map<K>(keys[i], (K)opos, (K)oneg);
        o |= t;
        a &= t;
    }
    for (int off = 32; off > 0; off >>= 1) {
        o |= __shfl_xor(o, off, 64);
        a &= __shfl_xor(a, off, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        atomicOr(&acc[0], (unsigned long long)o);
        atomicAnd(&acc[1], (unsigned long long)a);
    }
}

// mapped key bits from `s` up (0 when s reaches the key's width)
__device__ __forceinline__ uint64_t bits_from(uint64_t m, int s) { return s >= 64 ? 0ull : m >> s; }

// compressed 2^16-bin histogram (hist16_add) of the window bits [wshift,
// wshift + 16) & wmask of the keys whose bits from pshift up equal prefix
template <typename K>
__global__ __launch_bounds__(kHostThreads) void k_hist_window(const K* __restrict__ keys, uint64_t n, int wshift,
                                                              uint32_t wmask, int pshift, uint64_t prefix,
                                                              uint32_t* __restrict__ part, uint32_t* wrap_lo,
                                                              uint32_t* wrap_word, uint64_t opos, uint64_t oneg) {
    __shared__ uint32_t cnt[kHist16Words];
    for (int i = threadIdx.x; i < kHist16Words; i += kHostThreads) cnt[i] = 0;
    __syncthreads();
    const uint64_t stride = (uint64_t)gridDim.x * kHostThreads;
    for (uint64_t i = (uint64_t)blockIdx.x * kHostThreads + threadIdx.x; i < n; i += stride) {
        const uint64_t m = (uint64_t)order_map<K>(keys[i], (K)opos, (K)oneg);
        const bool in = bits_from(m, pshift) == prefix;
        hist16_add(cnt, in ? (uint32_t)(m >> wshift) & wmask : 0u, in ? 1u : 0u, wrap_lo, wrap_word);
    }
    __syncthreads();
    uint32_t* dst = part + (uint64_t)blockIdx.x * kHist16Words;
    for (int i = threadIdx.x; i < kHist16Words; i += kHostThreads) dst[i] = cnt[i];
}

// append the keys whose bits from pshift up equal prefix and whose window
// value lies in [lo, hi) to out (order within a range does not matter: equal
// keys are equal bits).  Each block counts the matches of its contiguous
// chunk, reserves that many slots with one atomic, then writes them (a
// second read of the chunk, from device memory).
template <typename K>
__global__ __launch_bounds__(kHostThreads) void k_select_range(const K* __restrict__ keys, uint64_t n, int wshift,
                                                               uint32_t wmask, int pshift, uint64_t prefix,
                                                               uint32_t lo, uint32_t hi, K* __restrict__ out,
                                                               uint64_t cap, unsigned long long* count,
                                                               uint32_t* err, uint64_t opos, uint64_t oneg) {
    __shared__ unsigned long long s_base;
    __shared__ uint32_t s_cnt;
    const uint64_t per = (n + gridDim.x - 1) / gridDim.x;
    const uint64_t c0 = (uint64_t)blockIdx.x * per, c1 = c0 + per < n ? c0 + per : n;
    auto in_range = [&](K k) {
        const uint64_t m = (uint64_t)order_map<K>(k, (K)opos, (K)oneg);
        const uint32_t v = (uint32_t)(m >> wshift) & wmask;
        return bits_from(m, pshift) == prefix && v >= lo && v < hi;
    };
    if (threadIdx.x == 0) s_cnt = 0;
    __syncthreads();
    uint32_t mine = 0;
    for (uint64_t i = c0 + threadIdx.x; i < c1; i += kHostThreads) mine += in_range(keys[i]) ? 1u : 0u;
    for (int off = 32; off > 0; off >>= 1) mine += __shfl_xor(mine, off, 64);
    if ((threadIdx.x & 63) == 0 && mine) atomicAdd(&s_cnt, mine);
    __syncthreads();
    if (threadIdx.x == 0) {
        s_base = s_cnt ? atomicAdd(count, (unsigned long long)s_cnt) : 0ull;
        s_cnt = 0;
    }
    __syncthreads();
    const unsigned long long base = s_base;
    for (uint64_t i0 = c0; i0 < c1; i0 += kHostThreads) {
        const uint64_t i = i0 + threadIdx.x;
        const K k = i < c1 ? keys[i] : (K)0;
        const bool take = i < c1 && in_range(k);
        const uint64_t m = ballot(take);
        if (m == 0) continue;
        uint32_t wbase = 0;
        if (lanes_below(m) == 0 && take) wbase = atomicAdd(&s_cnt, (uint32_t)popc64(m));
        wbase = __shfl(wbase, __builtin_ctzll(m), 64);
        if (take) {
            const uint64_t j = base + wbase + lanes_below(m);
            if (j < cap) out[j] = k;
            else atomicOr(err, 128u);  // more keys than the histogram counted
        }
    }
}

uint32_t host_grid(uint64_t n) {
    const uint64_t g = (n + kHostThreads - 1) / kHostThreads;
    const uint64_t cap = 4ull * (uint64_t)device_cu_count();
    return (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(g, cap));
}

}  // namespace
}  // namespace fs

extern "C" {

fs_status fs_sort_host(const void* h_keys_in, void* h_keys_out, uint64_t n, int key_bits, uint64_t batch_keys,
                       uint64_t device_keys, unsigned flags, void* workspace, size_t* workspace_bytes,
                       void* copy_stream, void* compute_stream) {
    using namespace fs;
    if (key_bits != 32 && key_bits != 64) return FS_ERR_INVALID_ARG;
    uint64_t opos, oneg;
    if (!order_masks(flags, key_bits, &opos, &oneg)) return FS_ERR_INVALID_ARG;
    if (!workspace_bytes || n > kMaxStreamKeys || batch_keys == 0 || batch_keys > kMaxStreamKeys ||
        device_keys == 0 || device_keys > kMaxStreamKeys)
        return FS_ERR_INVALID_ARG;
    const int kb = key_bits / 8;
    const uint64_t batch = (batch_keys + 3) / 4 * 4;
    size_t inner = 0;
    if (fs_sort_keys(nullptr, nullptr, device_keys, key_bits, 0, nullptr, &inner, nullptr) != FS_OK)
        return FS_ERR_INVALID_ARG;
    const uint32_t groups = host_grid(batch);
    // layout: inner sort workspace first (word 0 is its error word), then
    // the histogram, the reductions, the histogram parts, the staging slots,
    // the range buffer and its sorted copy
    const size_t o_inner = 0;
    const size_t o_hist = align256(inner);
    const size_t o_acc = o_hist + align256(kHistBytes);
    const size_t o_part = o_acc + 256;
    const size_t o_wrap = o_part + align256(4ull * groups * kHist16Words);
    const size_t o_slot0 = o_wrap + align256(4ull * 2 * kHist16Words);
    const size_t slot = align256(batch * kb);
    const size_t o_range = o_slot0 + 2 * slot;
    const size_t o_sorted = o_range + align256(device_keys * kb);
    const size_t need = o_sorted + align256(device_keys * kb);
    if (!workspace) {
        *workspace_bytes = need;
        return FS_OK;
    }
    if (*workspace_bytes < need) return FS_ERR_WORKSPACE_TOO_SMALL;
    if ((n && (!h_keys_in || !h_keys_out)) || !aligned(workspace, 256) || (h_keys_in && !aligned(h_keys_in, kb)) ||
        (h_keys_out && !aligned(h_keys_out, kb)))
        return FS_ERR_INVALID_ARG;
    const uintptr_t ia = reinterpret_cast<uintptr_t>(h_keys_in), oa = reinterpret_cast<uintptr_t>(h_keys_out);
    if (n && ia < oa + n * kb && oa < ia + n * kb) return FS_ERR_INVALID_ARG;  // the input is read to the end
    if (n == 0) return FS_OK;

    hipStream_t cs = static_cast<hipStream_t>(compute_stream);
    hipStream_t xs = static_cast<hipStream_t>(copy_stream);
    char* ws = static_cast<char*>(workspace);
    uint32_t* err = reinterpret_cast<uint32_t*>(ws + o_inner);
    uint64_t* hist = reinterpret_cast<uint64_t*>(ws + o_hist);
    unsigned long long* acc = reinterpret_cast<unsigned long long*>(ws + o_acc);  // or, and, count
    uint32_t* serr = reinterpret_cast<uint32_t*>(acc + 3);  // selection's error word
    uint32_t* part = reinterpret_cast<uint32_t*>(ws + o_part);
    uint32_t* wrap = reinterpret_cast<uint32_t*>(ws + o_wrap);
    char* slots[2] = {ws + o_slot0, ws + o_slot0 + slot};
    char* range = ws + o_range;
    char* sorted = ws + o_sorted;
    const char* in = static_cast<const char*>(h_keys_in);
    char* out = static_cast<char*>(h_keys_out);
    const uint64_t batches = (n + batch - 1) / batch;

    SlotEvents ev;
    if (!ev.ok) return FS_ERR_DEVICE;
    // copies back to the host run on a stream of their own (default
    // priority), beside the next range's copies in
    struct OwnStream {
        hipStream_t s = nullptr;
        hipEvent_t sorted = nullptr, drained = nullptr;
        bool ok = hipStreamCreateWithFlags(&s, hipStreamNonBlocking) == hipSuccess &&
                  hipEventCreateWithFlags(&sorted, hipEventDisableTiming) == hipSuccess &&
                  hipEventCreateWithFlags(&drained, hipEventDisableTiming) == hipSuccess;
        ~OwnStream() {
            if (s) {
                (void)hipStreamSynchronize(s);
                (void)hipStreamDestroy(s);
            }
            if (sorted) (void)hipEventDestroy(sorted);
            if (drained) (void)hipEventDestroy(drained);
        }
    } back;
    if (!back.ok) return FS_ERR_DEVICE;
    bool ok = launch_fill_u32(err, 1, 0u, cs) == hipSuccess;
    // stream every batch through the two staging slots, running `work` on
    // each as it arrives (compute stream), then wait for the compute stream
    auto stream_input = [&](auto&& work) {
        for (uint64_t b = 0; ok && b < batches; ++b) {
            const int i = (int)(b & 1);
            const uint64_t off = b * batch, len = std::min(batch, n - off);
            if (b >= 2) ok = hipStreamWaitEvent(xs, ev.emptied[i], 0) == hipSuccess;
            ok = ok && hipMemcpyAsync(slots[i], in + off * kb, len * kb, hipMemcpyHostToDevice, xs) == hipSuccess;
            ok = ok && hipEventRecord(ev.filled[i], xs) == hipSuccess;
            ok = ok && hipStreamWaitEvent(cs, ev.filled[i], 0) == hipSuccess;
            ok = ok && work(slots[i], len);
            ok = ok && hipEventRecord(ev.emptied[i], cs) == hipSuccess;
        }
        ok = ok && hipStreamSynchronize(cs) == hipSuccess;
    };
    auto launch_ok = [&]() { return hipGetLastError() == hipSuccess; };

    // 1. the bits on which keys differ
    ok = ok && launch_fill_u32(reinterpret_cast<uint32_t*>(acc), 2, 0u, cs) == hipSuccess &&
         launch_fill_u32(reinterpret_cast<uint32_t*>(acc + 1), 2, 0xFFFFFFFFu, cs) == hipSuccess &&
         launch_fill_u32(serr, 1, 0u, cs) == hipSuccess;
    stream_input([&](const char* keys, uint64_t len) {
        if (kb == 4)
            k_or_and<uint32_t><<<host_grid(len), kHostThreads, 0, cs>>>((const uint32_t*)keys, len, acc, opos, oneg);
        else
            k_or_and<uint64_t><<<host_grid(len), kHostThreads, 0, cs>>>((const uint64_t*)keys, len, acc, opos, oneg);
        return launch_ok();
    });
    unsigned long long oa_h[2] = {0, 0};
    ok = ok && hipMemcpy(oa_h, acc, sizeof oa_h, hipMemcpyDeviceToHost) == hipSuccess;
    if (!ok) return FS_ERR_DEVICE;
    const uint64_t diff = oa_h[0] ^ oa_h[1];
    if (diff == 0) {  // every key is the same: the input is sorted
        std::memcpy(out, in, n * kb);
        return FS_OK;
    }
    const int top = 63 - __builtin_clzll(diff);
    const uint64_t all = key_bits == 64 ? ~0ull : (1ull << key_bits) - 1;
    // caller's bits of a mapped key value (the inverse of order_map)
    auto unmap = [&](uint64_t t) {
        const uint64_t sign = 1ull << (key_bits - 1);
        return (t ^ ((((t ^ oneg) & sign) != 0) ? oneg : opos)) & all;
    };
    auto shr = [](uint64_t x, int s) { return s >= 64 ? 0ull : x >> s; };

    // 2 and 3, for the keys whose mapped bits from pshift up equal prefix:
    // the 2^16-bin histogram of the 16 bits below pshift, then ranges of
    // consecutive window values that fit the device, in order, each gathered,
    // sorted and copied back; a bin holding more keys than the device takes
    // is split again by its next 16 bits, and at the lowest window such a bin
    // is one key value, written out as a run of it.  The first call covers
    // every key: the bits above the top differing bit are the same in all.
    std::vector<uint64_t> h(65536);
    uint64_t placed = 0;
    auto visit = [&](auto&& self, uint64_t prefix, int pshift) -> fs_status {
        const int wshift = pshift > 16 ? pshift - 16 : 0;
        const uint32_t wmask = (uint32_t)((1ull << (pshift - wshift)) - 1);
        ok = launch_fill_u32(reinterpret_cast<uint32_t*>(hist), 2 * 65536, 0, cs) == hipSuccess;
        stream_input([&](const char* keys, uint64_t len) {
            const uint32_t g = std::min<uint32_t>(groups, host_grid(len));
            if (launch_fill_u32(wrap, 2ull * kHist16Words, 0, cs) != hipSuccess) return false;
            if (kb == 4)
                k_hist_window<uint32_t><<<g, kHostThreads, 0, cs>>>((const uint32_t*)keys, len, wshift, wmask, pshift,
                                                                    prefix, part, wrap, wrap + kHist16Words, opos, oneg);
            else
                k_hist_window<uint64_t><<<g, kHostThreads, 0, cs>>>((const uint64_t*)keys, len, wshift, wmask, pshift,
                                                                    prefix, part, wrap, wrap + kHist16Words, opos, oneg);
            return launch_ok() && launch_merge16(part, g, wrap, wrap + kHist16Words, hist, cs, true) == hipSuccess;
        });
        ok = ok && hipMemcpy(h.data(), hist, kHistBytes, hipMemcpyDeviceToHost) == hipSuccess;
        if (!ok) return FS_ERR_DEVICE;
        std::vector<uint64_t> hv(h.begin(), h.begin() + (size_t)wmask + 1);  // h is reused below this level
        for (uint32_t v0 = 0; v0 <= wmask;) {
            if (hv[v0] > device_keys) {
                const uint64_t sub = (prefix << (pshift - wshift)) | v0;
                if (wshift == 0) {
                    // one key value: its run goes straight to the output
                    ok = hipStreamSynchronize(back.s) == hipSuccess;
                    if (!ok) return FS_ERR_DEVICE;
                    const uint64_t value = unmap(sub);
                    for (uint64_t i = 0; i < hv[v0]; ++i) {
                        if (kb == 4) reinterpret_cast<uint32_t*>(out)[placed + i] = (uint32_t)value;
                        else reinterpret_cast<uint64_t*>(out)[placed + i] = value;
                    }
                    placed += hv[v0];
                } else {
                    const fs_status st = self(self, sub, wshift);
                    if (st != FS_OK) return st;
                }
                ++v0;
                continue;
            }
            uint64_t cnt = 0;
            uint32_t v1 = v0;
            while (v1 <= wmask && hv[v1] <= device_keys && cnt + hv[v1] <= device_keys) cnt += hv[v1++];
            if (cnt) {
                ok = launch_fill_u32(reinterpret_cast<uint32_t*>(acc + 2), 2, 0u, cs) == hipSuccess;
                stream_input([&](const char* keys, uint64_t len) {
                    if (kb == 4)
                        k_select_range<uint32_t><<<host_grid(len), kHostThreads, 0, cs>>>(
                            (const uint32_t*)keys, len, wshift, wmask, pshift, prefix, v0, v1, (uint32_t*)range, cnt,
                            acc + 2, serr, opos, oneg);
                    else
                        k_select_range<uint64_t><<<host_grid(len), kHostThreads, 0, cs>>>(
                            (const uint64_t*)keys, len, wshift, wmask, pshift, prefix, v0, v1, (uint64_t*)range, cnt,
                            acc + 2, serr, opos, oneg);
                    return launch_ok();
                });
                unsigned long long got = 0;
                ok = ok && hipMemcpy(&got, acc + 2, sizeof got, hipMemcpyDeviceToHost) == hipSuccess;
                if (!ok || got != cnt) return FS_ERR_DEVICE;
                // the previous range's copy back must have left the sorted buffer
                ok = hipStreamWaitEvent(cs, back.drained, 0) == hipSuccess;
                size_t ib = inner;
                if (!ok || fs_sort_keys(range, sorted, cnt, key_bits, flags, ws + o_inner, &ib, cs) != FS_OK)
                    return FS_ERR_DEVICE;
                uint32_t e = 0;  // the range sort's error word
                ok = hipEventRecord(back.sorted, cs) == hipSuccess &&
                     hipStreamWaitEvent(back.s, back.sorted, 0) == hipSuccess &&
                     hipMemcpyAsync(out + placed * kb, sorted, cnt * kb, hipMemcpyDeviceToHost, back.s) == hipSuccess &&
                     hipEventRecord(back.drained, back.s) == hipSuccess &&
                     hipStreamSynchronize(cs) == hipSuccess &&
                     hipMemcpy(&e, err, sizeof e, hipMemcpyDeviceToHost) == hipSuccess;
                if (!ok || e != 0) return FS_ERR_DEVICE;
                placed += cnt;
            }
            v0 = v1;
        }
        return FS_OK;
    };
    const int pshift0 = top + 1;  // bits from here up are common to every key
    const fs_status st = visit(visit, shr(oa_h[0], pshift0), pshift0);
    if (st != FS_OK) return st;
    uint32_t e = 0;
    ok = hipStreamSynchronize(back.s) == hipSuccess &&
         hipMemcpy(&e, serr, sizeof e, hipMemcpyDeviceToHost) == hipSuccess;
    return ok && e == 0 && placed == n ? FS_OK : FS_ERR_DEVICE;
}

}  // extern "C"
