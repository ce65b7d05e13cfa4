// Histogram, merge, prefix-scan, plan and expansion kernels.
//
// The histogram follows the paper's compressed tree of counters (Section
// III-B.1 Fractal RMW, Algorithm 1; counter width tapering, Section
// III-D.1).  For a d-bit digit the tree is complete and implicit (Algorithm
// 4: nodes at computable positions, no pointers), its leaves are the 2^d
// digit values and every inner node is the sum of its leaves, so a key
// updates only its leaf and the inner sums are produced by the prefix scan.
// The leaf counters are narrow: the 2^16-bin histogram of 16-bit keys keeps
// two 16-bit counters per 32-bit LDS word (128 KiB, which fits the 160 KiB
// LDS of a CDNA4 compute unit where 2^16 32-bit counters would not), and a
// counter that wraps is repaired exactly from side counts kept in global
// memory (see k_hist16c).
#include "fs_device.hpp"
#include "fs_internal.hpp"
#include "fs_plan.hpp"

namespace fs {

__global__ void k_fill_u32(uint32_t* p, uint64_t words, uint32_t value) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < words; i += stride)
        p[i] = value;
}

__global__ void k_zero(ZeroRanges r, uint64_t total) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += stride) {
        uint64_t j = i;
        int k = 0;
        while (j >= r.words[k]) j -= r.words[k++];  // total bounds i, so k stays below 4
        r.p[k][j] = 0;
    }
}

hipError_t launch_zero(const ZeroRanges& r, hipStream_t s) {
    const uint64_t total = r.words[0] + r.words[1] + r.words[2] + r.words[3];
    if (total == 0) return hipSuccess;
    uint64_t g = (total + 255) / 256;
    if (g > 8192) g = 8192;
    k_zero<<<(unsigned)g, 256, 0, s>>>(r, total);
    return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t* p, uint64_t words, uint32_t value, hipStream_t s) {
    if (words == 0) return hipSuccess;
    uint64_t g = (words + 255) / 256;
    if (g > 8192) g = 8192;
    k_fill_u32<<<(unsigned)g, 256, 0, s>>>(p, words, value);
    return hipGetLastError();
}

// ----------------------------------------------------------------------------
// Compressed 2^16-bin histogram of 16-bit keys, one per workgroup
// (hist16_add, fs_device.hpp).
// ----------------------------------------------------------------------------
// With ORD the mapped keys are counted (order_map with masks opos, oneg).
template <bool ORD>
__global__ __launch_bounds__(kHist16Threads) void k_hist16c(
    const uint16_t* __restrict__ keys, uint64_t n, uint64_t head, uint64_t nvec,
    uint32_t* __restrict__ part, uint32_t* wrap_lo, uint32_t* wrap_word, uint32_t opos, uint32_t oneg) {
    __shared__ uint32_t cnt[kHist16Words];
    const int tid = threadIdx.x;
    for (int i = tid; i < kHist16Words; i += kHist16Threads) cnt[i] = 0;
    __syncthreads();

    // contiguous chunk of 8-key vectors for this workgroup
    const uint64_t per = (nvec + gridDim.x - 1) / gridDim.x;
    const uint64_t v0 = (uint64_t)blockIdx.x * per;
    const uint64_t v1 = v0 + per < nvec ? v0 + per : nvec;
    const u32x4* vec = reinterpret_cast<const u32x4*>(keys + head);
    // kHist16Unroll vectors per thread are requested before any is counted,
    // so each thread keeps that many loads in flight (HBM latency, not the
    // LDS adds, bounds this loop otherwise)
    constexpr int U = kHist16Unroll;
    for (uint64_t v0u = v0 + tid; v0u < v1; v0u += (uint64_t)U * kHist16Threads) {
        u32x4 qs[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint64_t v = v0u + (uint64_t)u * kHist16Threads;
            qs[u] = __builtin_nontemporal_load(&vec[v < v1 ? v : v0u]);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint64_t v = v0u + (uint64_t)u * kHist16Threads;
            if (__builtin_amdgcn_readfirstlane((uint32_t)(v >= v1 ? 1u : 0u)) && v >= v1) break;  // wave-uniform tail
            const bool in = v < v1;
            u32x4 q = qs[u];
            if constexpr (ORD) q = order_map_vec<uint16_t>(q, opos, oneg);
            const uint32_t w[4] = {q.x, q.y, q.z, q.w};
            // whole wave holding one key value: one add for all of it
            const uint32_t k0 = w[0] & 0xFFFFu;
            const bool uniform_lane = in && (w[0] >> 16) == k0 && w[1] == w[0] && w[2] == w[0] && w[3] == w[0];
            const uint32_t kw = __builtin_amdgcn_readfirstlane(k0);
            const uint64_t active = ballot(in);
            const uint64_t same = ballot(uniform_lane && k0 == kw);
            if (same == active) {
                if (in && lanes_below(active) == 0)
                    hist16_add(cnt, kw, 8u * popc64(active), wrap_lo, wrap_word);
                continue;
            }
            // otherwise one add per run of equal keys within the lane (counted
            // at the run's last key, 0 elsewhere), all issued together; lanes
            // past the end add 0
            uint32_t k[8], c[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) k[e] = (w[e >> 1] >> (16 * (e & 1))) & 0xFFFFu;
            // no lane past the end and no two equal neighbours in any lane:
            // an add of one per key
            bool runs = !in;
#pragma unroll
            for (int e = 0; e < 7; ++e) runs |= k[e + 1] == k[e];
            if (ballot(runs) == 0) {
                hist16_add_ones<8>(cnt, k, nullptr, wrap_lo, wrap_word);
                continue;
            }
            uint32_t run = 1;
#pragma unroll
            for (int e = 0; e < 7; ++e) {
                const bool same_next = k[e + 1] == k[e];
                c[e] = (same_next || !in) ? 0u : run;
                run = same_next ? run + 1 : 1u;
            }
            c[7] = in ? run : 0u;
            hist16_add_n<8>(cnt, k, c, wrap_lo, wrap_word);
        }
    }
    // the few keys before the first 16-byte boundary and after the last vector
    if (blockIdx.x == 0) {
        const uint64_t tail0 = head + 8 * nvec;
        const uint64_t extra = head + (n - tail0);
        for (uint64_t e = tid; e < extra; e += kHist16Threads) {
            const uint64_t i = e < head ? e : tail0 + (e - head);
            const uint16_t k = ORD ? order_map<uint16_t>(keys[i], (uint16_t)opos, (uint16_t)oneg) : keys[i];
            hist16_add(cnt, k, 1u, wrap_lo, wrap_word);
        }
    }
    __syncthreads();
    uint32_t* dst = part + (uint64_t)blockIdx.x * kHist16Words;
    for (int i = tid; i < kHist16Words; i += kHist16Threads) dst[i] = cnt[i];
}

hipError_t launch_hist16c(const uint16_t* keys, uint64_t n, uint32_t groups, uint32_t* part,
                          uint32_t* wrap_lo, uint32_t* wrap_word, hipStream_t s, uint32_t opos, uint32_t oneg) {
    const uintptr_t a = reinterpret_cast<uintptr_t>(keys);
    uint64_t head = ((16 - (a & 15)) & 15) / 2;
    if (head > n) head = n;
    const uint64_t nvec = (n - head) / 8;
    if (opos | oneg)
        k_hist16c<true><<<groups, kHist16Threads, 0, s>>>(keys, n, head, nvec, part, wrap_lo, wrap_word, opos, oneg);
    else
        k_hist16c<false><<<groups, kHist16Threads, 0, s>>>(keys, n, head, nvec, part, wrap_lo, wrap_word, 0, 0);
    return hipGetLastError();
}

// Sum the per-workgroup packed counters and repair wraps -> exact uint64
// counts of all 2^16 bins (the global merge of Section III-A.1 / III-B).
// With `accumulate` the counts are added to h16 instead of replacing it: the
// histogram of a stream of batches is the sum of theirs (Section III-C).
// A block owns kMergeWords packed words; its eight 32-thread slices each sum
// every eighth workgroup's copy, so the loads of a word are spread over the
// whole GPU rather than queued in one thread.
constexpr int kMergeWords = 32;
constexpr int kMergeSlices = 8;

template <bool kAccumulate>
__global__ __launch_bounds__(kMergeWords * kMergeSlices) void k_merge16(
    const uint32_t* __restrict__ part, uint32_t groups, const uint32_t* __restrict__ wrap_lo,
    const uint32_t* __restrict__ wrap_word, uint64_t* __restrict__ h16) {
    __shared__ uint64_t s_lo[kMergeSlices][kMergeWords], s_all[kMergeSlices][kMergeWords];
    const int tid = threadIdx.x, wl = tid % kMergeWords, slice = tid / kMergeWords;
    const uint32_t w = blockIdx.x * kMergeWords + wl;
    uint64_t lo = 0, all = 0;
#pragma unroll 4
    for (uint32_t g = slice; g < groups; g += kMergeSlices) {
        const uint32_t x = part[(uint64_t)g * kHist16Words + w];
        lo += x & 0xFFFFu;
        all += x;
    }
    s_lo[slice][wl] = lo;
    s_all[slice][wl] = all;
    __syncthreads();
    if (tid < kMergeWords) {
        lo = 0;
        all = 0;
#pragma unroll
        for (int k = 0; k < kMergeSlices; ++k) {
            lo += s_lo[k][tid];
            all += s_all[k][tid];
        }
        lo += (uint64_t)wrap_lo[w] << 16;
        all += (uint64_t)wrap_word[w] << 32;
        const uint64_t hi = (all - lo) >> 16;
        if (kAccumulate) {
            h16[2 * w] += lo;
            h16[2 * w + 1] += hi;
        } else {
            h16[2 * w] = lo;
            h16[2 * w + 1] = hi;
        }
    }
}

hipError_t launch_merge16(const uint32_t* part, uint32_t groups, const uint32_t* wrap_lo,
                          const uint32_t* wrap_word, uint64_t* h16, hipStream_t s, bool accumulate) {
    constexpr unsigned blocks = kHist16Words / kMergeWords, threads = kMergeWords * kMergeSlices;
    if (accumulate)
        k_merge16<true><<<blocks, threads, 0, s>>>(part, groups, wrap_lo, wrap_word, h16);
    else
        k_merge16<false><<<blocks, threads, 0, s>>>(part, groups, wrap_lo, wrap_word, h16);
    return hipGetLastError();
}

// Exclusive prefix of the 2^16 bins (GetIndex of every value, Algorithm 3):
// p16[v] = sum(h16[0..v-1]), p16[65536] = n.  Block b of kScanBlocks owns
// bins [1024 b, 1024 b + 1024), one per thread; it sums all bins before its
// own (the whole histogram is 512 KiB and is read from L2), then scans its
// own bins.  No block waits for another.
constexpr int kScanThreads = 1024;
constexpr int kScanBlocks = 65536 / kScanThreads;

// exclusive scan of one value per thread over a block of kScanThreads; *total gets the sum
__device__ __forceinline__ uint64_t scan_block1024(uint64_t x, uint64_t* wsum, uint64_t* total) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    uint64_t inc = x;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint64_t y = __shfl_up(inc, off, 64);
        if (lane >= off) inc += y;
    }
    if (lane == 63) wsum[wave] = inc;
    __syncthreads();
    uint64_t before = 0, all = 0;
#pragma unroll
    for (int w = 0; w < kScanThreads / 64; ++w) {
        const uint64_t v = wsum[w];
        if (w < wave) before += v;
        all += v;
    }
    *total = all;
    return before + inc - x;
}

__global__ __launch_bounds__(kScanThreads) void k_scan16(const uint64_t* __restrict__ h16,
                                                         uint64_t* __restrict__ p16) {
    __shared__ uint64_t wsum[kScanThreads / 64];
    __shared__ uint64_t wsum2[kScanThreads / 64];
    const int tid = threadIdx.x;
    const uint32_t b = blockIdx.x;
    // sum of the bins of all earlier blocks
    uint64_t acc = 0;
#pragma unroll 4
    for (uint32_t i = tid; i < b * kScanThreads; i += kScanThreads) acc += h16[i];
    uint64_t base;
    (void)scan_block1024(acc, wsum, &base);
    // this block's bins
    const uint32_t v = b * kScanThreads + tid;
    const uint64_t c = h16[v];
    uint64_t total;
    const uint64_t excl = scan_block1024(c, wsum2, &total);
    p16[v] = base + excl;
    if (v == 65535) p16[65536] = base + total;
}

hipError_t launch_scan16(const uint64_t* h16, uint64_t* p16, hipStream_t s) {
    k_scan16<<<kScanBlocks, kScanThreads, 0, s>>>(h16, p16);
    return hipGetLastError();
}

// Digit histograms of 16-bit keys as marginals of the 2^16-bin histogram:
// digit 0 (low byte) sums each column, digit 1 (high byte) each row.
__global__ __launch_bounds__(256) void k_plan_from16(const uint64_t* __restrict__ h16, uint64_t n,
                                                     uint64_t* hist, uint64_t* base, uint32_t* plan,
                                                     bool clobber) {
    const int b = threadIdx.x;
    uint64_t h[2] = {0, 0};
    for (int i = 0; i < 256; ++i) {
        h[0] += h16[i * 256 + b];
        h[1] += h16[b * 256 + i];
    }
    finish_plan(h, 2, n, hist, base, plan, clobber);
}

hipError_t launch_plan_from16(const uint64_t* h16, uint64_t n, uint64_t* hist, uint64_t* base,
                              uint32_t* plan, hipStream_t s, bool clobber) {
    k_plan_from16<<<1, 256, 0, s>>>(h16, n, hist, base, plan, clobber);
    return hipGetLastError();
}

// ----------------------------------------------------------------------------
// Per-workgroup 8-bit digit histograms of all digits in one read of the keys.
// part[g][j][b] = count of digit j == b among workgroup g's keys.
// ----------------------------------------------------------------------------
template <typename K>
__global__ __launch_bounds__(kHist8Threads) void k_hist8(const K* __restrict__ keys, uint64_t n,
                                                         uint64_t head, uint64_t nvec,
                                                         uint32_t* __restrict__ part) {
    constexpr int D = sizeof(K);
    constexpr int VK = 16 / sizeof(K);
    __shared__ uint32_t cnt[D][kRadix];
    const int tid = threadIdx.x;
    for (int i = tid; i < D * kRadix; i += kHist8Threads) (&cnt[0][0])[i] = 0;
    __syncthreads();
    const uint64_t per = (nvec + gridDim.x - 1) / gridDim.x;
    const uint64_t v0 = (uint64_t)blockIdx.x * per;
    const uint64_t v1 = v0 + per < nvec ? v0 + per : nvec;
    const u32x4* vec = reinterpret_cast<const u32x4*>(keys + head);
    for (uint64_t v = v0 + tid; v < v1; v += kHist8Threads) {
        const u32x4 q = __builtin_nontemporal_load(&vec[v]);
        K k[VK];
        __builtin_memcpy(k, &q, 16);
        bool lane_same = true;
#pragma unroll
        for (int e = 1; e < VK; ++e) lane_same &= k[e] == k[0];
        const uint64_t active = ballot(true);
        const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)(uint64_t)k[0]);
        const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)k[0] >> 32));
        const uint64_t kw = ((uint64_t)hi << 32) | lo;
        if (ballot(lane_same && (uint64_t)k[0] == kw) == active) {
            if (lanes_below(active) == 0) {
#pragma unroll
                for (int j = 0; j < D; ++j)
                    atomicAdd(&cnt[j][digit_of<uint64_t>(kw, 8 * j)], (uint32_t)VK * popc64(active));
            }
            continue;
        }
#pragma unroll
        for (int e = 0; e < VK; ++e) {
#pragma unroll
            for (int j = 0; j < D; ++j) atomicAdd(&cnt[j][digit_of<K>(k[e], 8 * j)], 1u);
        }
    }
    if (blockIdx.x == 0) {
        const uint64_t tail0 = head + (uint64_t)VK * nvec;
        const uint64_t extra = head + (n - tail0);
        for (uint64_t e = tid; e < extra; e += kHist8Threads) {
            const K key = keys[e < head ? e : tail0 + (e - head)];
#pragma unroll
            for (int j = 0; j < D; ++j) atomicAdd(&cnt[j][digit_of<K>(key, 8 * j)], 1u);
        }
    }
    __syncthreads();
    uint32_t* dst = part + (uint64_t)blockIdx.x * D * kRadix;
    for (int i = tid; i < D * kRadix; i += kHist8Threads) dst[i] = (&cnt[0][0])[i];
}

hipError_t launch_hist8(const void* keys, uint64_t n, int key_bytes, uint32_t groups,
                        uint32_t* part, hipStream_t s) {
    const uintptr_t a = reinterpret_cast<uintptr_t>(keys);
    uint64_t head = ((16 - (a & 15)) & 15) / key_bytes;
    if (head > n) head = n;
    const uint64_t nvec = (n - head) / (16 / key_bytes);
    switch (key_bytes) {
    case 2: k_hist8<uint16_t><<<groups, kHist8Threads, 0, s>>>((const uint16_t*)keys, n, head, nvec, part); break;
    case 4: k_hist8<uint32_t><<<groups, kHist8Threads, 0, s>>>((const uint32_t*)keys, n, head, nvec, part); break;
    default: k_hist8<uint64_t><<<groups, kHist8Threads, 0, s>>>((const uint64_t*)keys, n, head, nvec, part); break;
    }
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_plan8(const uint32_t* __restrict__ part, uint32_t groups,
                                               int digits, uint64_t n, uint64_t* hist,
                                               uint64_t* base, uint32_t* plan) {
    const int b = threadIdx.x;
    uint64_t h[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (uint32_t g = 0; g < groups; ++g) {
        const uint32_t* p = part + (uint64_t)g * digits * kRadix;
        for (int j = 0; j < digits; ++j) h[j] += p[j * kRadix + b];
    }
    finish_plan(h, digits, n, hist, base, plan);
}

hipError_t launch_plan8(const uint32_t* part, uint32_t groups, int digits, uint64_t n,
                        uint64_t* hist, uint64_t* base, uint32_t* plan, hipStream_t s) {
    k_plan8<<<1, 256, 0, s>>>(part, groups, digits, n, hist, base, plan);
    return hipGetLastError();
}

// Sum per-workgroup digit histograms into uint64 counts (no plan).
__global__ __launch_bounds__(256) void k_reduce8(const uint32_t* __restrict__ part, uint32_t groups,
                                                 int digits, uint64_t* __restrict__ hist) {
    const int j = blockIdx.x, b = threadIdx.x;
    uint64_t h = 0;
    for (uint32_t g = 0; g < groups; ++g) h += part[((uint64_t)g * digits + j) * kRadix + b];
    hist[j * kRadix + b] = h;
}

hipError_t launch_reduce8(const uint32_t* part, uint32_t groups, int digits, uint64_t* hist,
                          hipStream_t s) {
    k_reduce8<<<digits, 256, 0, s>>>(part, groups, digits, hist);
    return hipGetLastError();
}

// ----------------------------------------------------------------------------
// Keys-only 16-bit sort written straight from the histogram (Algorithm 5
// with no trailing bits): out[i] = v for p16[v] <= i < p16[v+1].  Each
// workgroup owns 8192 output slots; it finds the value at its first and last
// slot by an order-statistic search of the prefix (GetItem, Algorithm 2),
// then every thread writes 8 consecutive keys with one 16-byte store.
// ----------------------------------------------------------------------------
constexpr int kExpandThreads = 256;
constexpr int kExpandGroupsPerThread = 4;
constexpr int kExpandSpan = kExpandThreads * 8 * kExpandGroupsPerThread;

// largest v in [lo, hi] with p[v] <= pos (p non-decreasing, p[lo] <= pos)
__device__ __forceinline__ uint32_t value_at(const uint64_t* p, uint32_t lo, uint32_t hi, uint64_t pos) {
    while (lo < hi) {
        const uint32_t mid = (lo + hi + 1) >> 1;
        if (p[mid] <= pos) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Sorted positions [first, first + count) of the multiset whose exclusive
// prefix is p16 (p16[65536] = total): position i holds the value v with
// p16[v] <= i < p16[v + 1] (Algorithm 5 with no trailing bits, i.e. the
// keys rebuilt from the leaf counters alone).  out[i - first] receives
// position i; positions at or past the total are not written.  With ORD
// the histogram counts mapped keys and each value is unmapped as it is
// written (order_unmap with masks opos, oneg).
// value_at over all 2^16 bins by one wave: each round the 64 lanes probe
// evenly spaced bins and the interval shrinks 64-fold (3 rounds of parallel
// loads instead of 16 dependent ones).  Every lane returns the result.
__device__ __forceinline__ uint32_t value_at_wave(const uint64_t* p, uint64_t pos) {
    const uint32_t lane = threadIdx.x & 63;
    uint32_t lo = 0, len = 65536;  // the answer is in [lo, lo + len); p[lo] <= pos
    while (len > 1) {
        const uint32_t step = (len + 63) / 64;
        const uint32_t idx = lo + lane * step;
        const bool ok = idx < lo + len && p[idx] <= pos;
        const uint64_t m = ballot(ok);  // lane 0 always holds (p[lo] <= pos); ok is monotone in lane
        const uint32_t last = 63 - (uint32_t)__builtin_clzll(m);
        lo += last * step;
        const uint32_t rest = lo + step < 65536u ? step : 65536u - lo;
        len = rest < len ? rest : len;
    }
    return lo;
}

template <bool kVec, bool ORD>
__global__ __launch_bounds__(kExpandThreads) void k_expand16(const uint64_t* __restrict__ p16,
                                                             uint16_t* __restrict__ out, uint64_t first,
                                                             uint64_t count, uint32_t opos, uint32_t oneg) {
    __shared__ uint32_t window[2];
    const uint64_t total = p16[65536];
    const uint64_t end = first + count < total ? first + count : total;
    const uint64_t rs = first + (uint64_t)blockIdx.x * kExpandSpan;
    if (rs >= end) return;
    const uint64_t re = rs + kExpandSpan < end ? rs + kExpandSpan : end;
    // the block's first and last values: wave 0 and wave 1 search at once
    if (threadIdx.x < 128) {
        const uint32_t v = value_at_wave(p16, threadIdx.x < 64 ? rs : re - 1);
        if ((threadIdx.x & 63) == 0) window[threadIdx.x >> 6] = v;
    }
    __syncthreads();
    const uint32_t vlo = window[0], vhi = window[1];
#pragma unroll
    for (int u = 0; u < kExpandGroupsPerThread; ++u) {
        const uint64_t p0 = rs + ((uint64_t)u * kExpandThreads + threadIdx.x) * 8;
        if (p0 >= re) break;
        uint32_t v = value_at(p16, vlo, vhi, p0);
        uint64_t next = p16[v + 1];
        uint32_t o[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const uint64_t pos = p0 + e < end ? p0 + e : end - 1;
            while (next <= pos) {  // p16[65536] = total > pos, so v stays <= 65535
                ++v;
                next = p16[v + 1];
            }
            o[e] = ORD ? order_unmap<uint16_t>((uint16_t)v, (uint16_t)opos, (uint16_t)oneg) : v;
        }
        uint16_t* dst = out + (p0 - first);
        if (kVec && p0 + 8 <= end) {
            u32x4 q;
            q.x = o[0] | (o[1] << 16);
            q.y = o[2] | (o[3] << 16);
            q.z = o[4] | (o[5] << 16);
            q.w = o[6] | (o[7] << 16);
            __builtin_nontemporal_store(q, reinterpret_cast<u32x4*>(dst));
        } else {
            for (int e = 0; e < 8 && p0 + e < end; ++e) dst[e] = (uint16_t)o[e];
        }
    }
}

hipError_t launch_expand16(const uint64_t* p16, uint16_t* out, uint64_t first, uint64_t count, hipStream_t s,
                           uint32_t opos, uint32_t oneg) {
    if (count == 0) return hipSuccess;
    const unsigned groups = (unsigned)((count + kExpandSpan - 1) / kExpandSpan);
    const bool vec = (reinterpret_cast<uintptr_t>(out) & 15) == 0;
    if (opos | oneg) {
        if (vec) k_expand16<true, true><<<groups, kExpandThreads, 0, s>>>(p16, out, first, count, opos, oneg);
        else k_expand16<false, true><<<groups, kExpandThreads, 0, s>>>(p16, out, first, count, opos, oneg);
    } else {
        if (vec) k_expand16<true, false><<<groups, kExpandThreads, 0, s>>>(p16, out, first, count, 0, 0);
        else k_expand16<false, false><<<groups, kExpandThreads, 0, s>>>(p16, out, first, count, 0, 0);
    }
    return hipGetLastError();
}

// Copy src -> dst when the plan found every digit trivial (the sorted
// result is then the input itself).
template <typename W>
__global__ void k_copy_if(const uint32_t* plan, int word, const W* __restrict__ src, W* __restrict__ dst,
                          uint64_t words) {
    if (!plan[word]) return;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < words; i += stride)
        dst[i] = src[i];
}

hipError_t launch_copy_if(const uint32_t* plan, const void* src, void* dst, uint64_t bytes,
                          hipStream_t s, int word) {
    if (bytes == 0) return hipSuccess;
    const uintptr_t m = reinterpret_cast<uintptr_t>(src) | reinterpret_cast<uintptr_t>(dst) | bytes;
    auto grid = [](uint64_t words) { uint64_t g = (words + 255) / 256; return (unsigned)(g > 8192 ? 8192 : g); };
    if ((m & 15) == 0) k_copy_if<uint4><<<grid(bytes / 16), 256, 0, s>>>(plan, word, (const uint4*)src, (uint4*)dst, bytes / 16);
    else if ((m & 3) == 0) k_copy_if<uint32_t><<<grid(bytes / 4), 256, 0, s>>>(plan, word, (const uint32_t*)src, (uint32_t*)dst, bytes / 4);
    else if ((m & 1) == 0) k_copy_if<uint16_t><<<grid(bytes / 2), 256, 0, s>>>(plan, word, (const uint16_t*)src, (uint16_t*)dst, bytes / 2);
    else k_copy_if<uint8_t><<<grid(bytes), 256, 0, s>>>(plan, word, (const uint8_t*)src, (uint8_t*)dst, bytes);
    return hipGetLastError();
}

}  // namespace fs
