// Batched segmented sort: many independent segments in one call.
//
// The paper processes its input as batches that each update the histogram
// and are handled serially or in parallel (Sections III-C, IV-D); here a
// batch is a caller segment and every segment gets exactly the result a
// stand-alone sort would give it.  Segment descriptors live in device
// memory, so the whole schedule is decided on the device:
//   1. classify: each segment goes to one bin by width and length (bounds
//      from the launch tuning, fs_seg_tuning): the wave bin (at most 64
//      keys), the 16-bit-digit bin (16-bit keys without payload, long
//      enough), the LDS bin (short enough to fit in one workgroup's LDS), the
//      one-workgroup bin or the large bin of its (key, value) class;
//   1a. wave bin: one wave per segment ranks its keys in registers (k_seg_wave);
//   2. 16-bit-digit bin: the segment's compressed 2^16-bin histogram is
//      built in LDS and the sorted keys are written from it (one read and one
//      write of HBM, no scatter); one workgroup per medium segment, 2^18-key
//      parts of a long one on several;
//   3. LDS bin: persistent workgroups pop the queue and sort each segment
//      with 8-bit digits entirely in LDS (one read and one write of HBM);
//   4. one-workgroup bin, per width class: a workgroup sorts a whole segment
//      with 8-bit digits through global memory, walking its tiles in order;
//   5. large bin, per width class: tile layout, per-segment digit
//      histograms (one read), per-segment prefix scans and pass plans, then
//      one single-sweep scatter launch per digit over the tiles of all large
//      segments of the class at once, with decoupled look-back confined to
//      each segment.  Look-back state words carry an epoch (class, pass), so
//      they are cleared once per call rather than once per pass.
#include "fs_sort.h"
#include "fs_device.hpp"
#include "fs_internal.hpp"

namespace fs {

__host__ __device__ inline int seg_class(int kb, int vb) {
    return (kb == 2 ? 0 : kb == 4 ? 1 : 2) * 3 + (vb == 0 ? 0 : vb == 4 ? 1 : 2);
}
// keys of a small segment fill the front of an LDS buffer, payloads start at
// the next 16-byte boundary
__host__ __device__ inline uint32_t small_cap(int kb, int vb) { return (kSegSmallBytes - 16) / (uint32_t)(kb + vb); }
__host__ __device__ inline uint32_t small_val_offset(uint32_t cap, int kb) { return (cap * kb + 15u) & ~15u; }

// state word of a segment tile: epoch (7 bits) | flag (2 bits) | count (23 bits)
constexpr uint32_t kSegCountBits = 23;
constexpr uint32_t kSegCountMask = (1u << kSegCountBits) - 1;
constexpr uint32_t kSegAgg = 1u << kSegCountBits;
constexpr uint32_t kSegPrefix = 2u << kSegCountBits;

// counters (ctr[]): small count, small taken, per class: large count, tiles,
// one ticket per (class, pass); the 16-bit-digit and one-workgroup queues
__host__ __device__ inline int ctr_large(int c) { return 2 + c; }
__host__ __device__ inline int ctr_tiles(int c) { return 16 + c; }
__host__ __device__ inline int ctr_ticket(int c, int j) { return 32 + 8 * c + j; }
__host__ __device__ inline int ctr_seen() { return 119; }  // 64-bit running total of queued keys (8-byte aligned)
__host__ __device__ inline int ctr_expand_long() { return 121; }  // 16-bit-digit bin: long segments queued
__host__ __device__ inline int ctr_expand_rest() { return 122; }  //   other segments queued
__host__ __device__ inline int ctr_expand_taken() { return 123; }
__host__ __device__ inline int ctr_x16_parts() { return 124; }  // parts of the long segments
__host__ __device__ inline int ctr_wg(int c) { return 128 + c; }        // one-workgroup large segments queued
__host__ __device__ inline int ctr_wg_taken(int c) { return 137 + c; }  //   and taken
__host__ __device__ inline int ctr_wg_tmp(int c) { return 147 + 2 * c; }  // 64-bit temporary-pool bump (8-byte aligned)
__host__ __device__ inline int ctr_wave() { return 166; }        // wave-bin segments queued
__host__ __device__ inline int ctr_wave_taken() { return 167; }  //   and taken

// ---------------------------------------------------------------------------
// Key order of the call (order_map, fs_device.hpp): the kernels that touch
// keys have an ORD instantiation, launched when x.ord is set, which maps keys
// where they are loaded and unmaps them where they are stored; the other
// instantiation passes keys through untouched.
template <bool ORD, typename K>
__device__ __forceinline__ K seg_map(const SegCtx& x, K k) {
    constexpr int w = sizeof(K) == 2 ? 0 : sizeof(K) == 4 ? 1 : 2;
    if constexpr (ORD) return order_map<K>(k, (K)x.ord_pos[w], (K)x.ord_neg[w]);
    else return k;
}
template <bool ORD, typename K>
__device__ __forceinline__ K seg_unmap(const SegCtx& x, K t) {
    constexpr int w = sizeof(K) == 2 ? 0 : sizeof(K) == 4 ? 1 : 2;
    if constexpr (ORD) return order_unmap<K>(t, (K)x.ord_pos[w], (K)x.ord_neg[w]);
    else return t;
}

__global__ void k_seg_classify(SegCtx x) {
    for (uint32_t s = blockIdx.x * blockDim.x + threadIdx.x; s < x.nseg; s += gridDim.x * blockDim.x) {
        const fs_segment d = x.segs[s];
        if (d.n == 0) continue;
        const bool ok = (d.key_bits == 16 || d.key_bits == 32 || d.key_bits == 64) &&
                        (d.val_bytes == 0 || d.val_bytes == 4 || d.val_bytes == 8) && d.keys_in &&
                        d.keys_out && (d.val_bytes == 0 || (d.vals_in && d.vals_out)) && d.n <= x.max_seg;
        if (!ok) {
            atomicOr(x.err, 16u);
            continue;
        }
        // every size-derived workspace bound assumes the declared total_keys:
        // keys past it are refused (and flagged) rather than queued
        unsigned long long* seen = reinterpret_cast<unsigned long long*>(&x.ctr[ctr_seen()]);
        const unsigned long long before = atomicAdd(seen, (unsigned long long)d.n);
        if (before + d.n > x.total_keys) {
            atomicOr(x.err, 32u);
            continue;
        }
        const int kb = d.key_bits / 8, vb = d.val_bytes;
        if (d.n <= kSegWaveMaxKeys) {  // one wave sorts it in registers
            x.wave_list[atomicAdd(&x.ctr[ctr_wave()], 1u)] = s;
            continue;
        }
        const uint32_t small_max = x.small_max[kb == 2 ? 0 : kb == 4 ? 1 : 2];
        if (kb == 2 && vb == 0 && d.n >= x.expand_min) {
            // long segments (split over several workgroups) at the front
            if (d.n >= x.split_min) {
                x.expand_list[atomicAdd(&x.ctr[ctr_expand_long()], 1u)] = s;
            } else {
                x.expand_list[x.nseg - 1 - atomicAdd(&x.ctr[ctr_expand_rest()], 1u)] = s;
            }
        } else if (d.n <= small_cap(kb, vb) && d.n <= small_max) {
            const uint32_t i = atomicAdd(&x.ctr[0], 1u);
            x.small_list[i] = s;
        } else if (d.n <= x.wg_max) {
            const int c = seg_class(kb, vb);
            const uint32_t i = atomicAdd(&x.ctr[ctr_wg(c)], 1u);
            x.wg_list[(uint64_t)c * x.nseg + i] = s;
        } else {
            const int c = seg_class(kb, vb);
            const uint32_t i = atomicAdd(&x.ctr[ctr_large(c)], 1u);
            x.large_list[(uint64_t)c * x.nseg + i] = s;
        }
    }
}

// ---------------------------------------------------------------------------
// Small segments: LSD passes entirely in LDS.
// ---------------------------------------------------------------------------
constexpr int kSmallThreads = 256;
constexpr int kSmallItems = 8;
constexpr int kSmallWaves = kSmallThreads / kWave;

struct SmallShared {
    __attribute__((aligned(16))) unsigned char buf[2][kSegSmallBytes];
    uint64_t peers[kSmallWaves][kRadix];
    uint32_t wcnt[kSmallWaves][kRadix];
    uint32_t hist[kRadix];
    uint32_t run[kRadix];
    uint64_t wsum[4];
    uint32_t flag;
    uint32_t seg, next;
};

// Copy n elements from global memory into LDS, and back, with aligned
// 16-byte accesses: elements outside [0, n) of a global block are masked on
// loads (an aligned 16-byte block never leaves a mapped page) and partial
// blocks at either end are stored element by element.
template <typename T, int NT>
__device__ __forceinline__ void global_to_lds(const T* src, T* lds, uint32_t n) {
    constexpr int VK = 16 / (int)sizeof(T);
    constexpr int U = 4;
    const uintptr_t p = reinterpret_cast<uintptr_t>(src);
    const uintptr_t a0 = p & ~(uintptr_t)15;
    const uint32_t lead = (uint32_t)((p - a0) / sizeof(T));
    const uint32_t nv = (lead + n + VK - 1) / VK;
    const gptr<const u32x4> vp = (gptr<const u32x4>)(a0);
    for (uint32_t i0 = 0; i0 < nv; i0 += U * NT) {
        u32x4 v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint32_t i = i0 + u * NT + threadIdx.x;
            v[u] = __builtin_nontemporal_load(&vp[i < nv ? i : nv - 1]);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint32_t i = i0 + u * NT + threadIdx.x;
            const T* ev = reinterpret_cast<const T*>(&v[u]);
#pragma unroll
            for (int e = 0; e < VK; ++e) {
                const int64_t idx = (int64_t)i * VK + e - lead;
                if (i < nv && idx >= 0 && idx < (int64_t)n) lds[idx] = ev[e];
            }
        }
    }
}

template <typename T, int NT>
__device__ __forceinline__ void lds_to_global(const T* lds, T* dst, uint32_t n) {
    constexpr int VK = 16 / (int)sizeof(T);
    const uintptr_t p = reinterpret_cast<uintptr_t>(dst);
    const uintptr_t a0 = p & ~(uintptr_t)15;
    const int64_t lead = (int64_t)((p - a0) / sizeof(T));
    const uint32_t nv = (uint32_t)((lead + n + VK - 1) / VK);
    for (uint32_t i = threadIdx.x; i < nv; i += NT) {
        const int64_t p0 = (int64_t)i * VK - lead;
        if (p0 >= 0 && p0 + VK <= (int64_t)n) {
            union {
                T e[VK];
                u32x4 v;
            } b;
#pragma unroll
            for (int e = 0; e < VK; ++e) b.e[e] = lds[p0 + e];
            __builtin_nontemporal_store(b.v, (gptr<u32x4>)(a0 + 16ull * i));
        } else {
            for (int e = 0; e < VK; ++e)
                if (p0 + e >= 0 && p0 + e < (int64_t)n) to_global(dst)[p0 + e] = lds[p0 + e];
        }
    }
}

template <typename K, typename V, bool ORD>
__device__ __forceinline__ void sort_small(const SegCtx& x, const fs_segment& d, SmallShared& sm) {
    constexpr bool kHasVals = !__is_same(V, NoVal);
    using VS = typename std::conditional<kHasVals, V, uint32_t>::type;
    constexpr int D = sizeof(K);
    constexpr int kb = sizeof(K), vb = kHasVals ? sizeof(VS) : 0;
    const uint32_t n = (uint32_t)d.n;
    const uint32_t cap = small_cap(kb, vb);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    // buffers are addressed by index into the shared array (not through a
    // table of pointers) so that every access compiles to an LDS instruction
    const uint32_t voff = small_val_offset(cap, kb);
    auto kbuf = [&](int c) { return reinterpret_cast<K*>(sm.buf[c]); };
    auto vbuf = [&](int c) { return reinterpret_cast<VS*>(sm.buf[c] + voff); };
    global_to_lds<K, kSmallThreads>(static_cast<const K*>(d.keys_in), kbuf(0), n);
    if constexpr (kHasVals) global_to_lds<VS, kSmallThreads>(static_cast<const VS*>(d.vals_in), vbuf(0), n);
    __syncthreads();
    if constexpr (ORD) {
        for (uint32_t i = tid; i < n; i += kSmallThreads) kbuf(0)[i] = seg_map<ORD, K>(x, kbuf(0)[i]);
        __syncthreads();
    }
    int cur = 0;
    for (int j = 0; j < D; ++j) {
        const int shift = 8 * j;
        if (tid < kRadix) sm.hist[tid] = 0;
        __syncthreads();
        for (uint32_t i = tid; i < n; i += kSmallThreads) atomicAdd(&sm.hist[digit_of<K>(kbuf(cur)[i], shift)], 1u);
        __syncthreads();
        const uint32_t h = tid < kRadix ? sm.hist[tid] : 0;
        const int trivial = __syncthreads_or(h == n);
        if (trivial) continue;  // identity under a stable scatter
        uint64_t tot;
        const uint32_t start = (uint32_t)scan256_exclusive<uint64_t>(h, sm.wsum, &tot);
        if (tid < kRadix) sm.run[tid] = start;
        // scatter cur -> 1-cur in sub-tiles, input order preserved
        constexpr uint32_t ST = kSmallThreads * kSmallItems;
        for (uint32_t base = 0; base < n; base += ST) {
            const uint32_t cnt = (n - base) < ST ? (n - base) : ST;
            const uint32_t wbase = (uint32_t)wave * kWave * kSmallItems;
            for (int i = 0; i < kRadix / kWave; ++i) sm.wcnt[wave][lane + kWave * i] = 0;
            __builtin_amdgcn_wave_barrier();
            K key[kSmallItems];
            uint32_t rank[kSmallItems];
#pragma unroll
            for (int k = 0; k < kSmallItems; ++k) {
                const uint32_t idx = wbase + k * kWave + lane;
                const bool valid = idx < cnt;
                key[k] = valid ? kbuf(cur)[base + idx] : (K)0;
                rank[k] = wave_rank(digit_of<K>(key[k], shift), valid, sm.peers[wave], sm.wcnt[wave]);
            }
            __syncthreads();
            if (tid < kRadix) {
                uint32_t r = sm.run[tid];
                for (int w = 0; w < kSmallWaves; ++w) {
                    const uint32_t c = sm.wcnt[w][tid];
                    sm.wcnt[w][tid] = r;
                    r += c;
                }
                sm.run[tid] = r;
            }
            __syncthreads();
#pragma unroll
            for (int k = 0; k < kSmallItems; ++k) {
                const uint32_t idx = wbase + k * kWave + lane;
                if (idx < cnt) {
                    const uint32_t pos = sm.wcnt[wave][digit_of<K>(key[k], shift)] + rank[k];
                    if (pos < n) {
                        kbuf(1 - cur)[pos] = key[k];
                        if constexpr (kHasVals) vbuf(1 - cur)[pos] = vbuf(cur)[base + idx];
                    }
                }
            }
            __syncthreads();
        }
        cur = 1 - cur;
    }
    if constexpr (ORD) {
        for (uint32_t i = tid; i < n; i += kSmallThreads) kbuf(cur)[i] = seg_unmap<ORD, K>(x, kbuf(cur)[i]);
        __syncthreads();
    }
    lds_to_global<K, kSmallThreads>(kbuf(cur), static_cast<K*>(d.keys_out), n);
    if constexpr (kHasVals) lds_to_global<VS, kSmallThreads>(vbuf(cur), static_cast<VS*>(d.vals_out), n);
    __syncthreads();
}

// ---------------------------------------------------------------------------
// Wave bin: segments of at most 64 keys, one per wave.  Lane i holds key i;
// its output position is the number of keys of the segment that sort
// before it (smaller keys, and equal keys of lower index: stable), counted
// over the wave's registers with shuffles.  No LDS, no barrier.
// ---------------------------------------------------------------------------
constexpr int kWaveThreads = 256;

__device__ __forceinline__ uint64_t load_elem(const void* p, uint32_t i, int bytes) {
    if (bytes == 2) return to_global(static_cast<const uint16_t*>(p))[i];
    if (bytes == 4) return to_global(static_cast<const uint32_t*>(p))[i];
    return to_global(static_cast<const uint64_t*>(p))[i];
}

__device__ __forceinline__ void store_elem(void* p, uint32_t i, int bytes, uint64_t v) {
    if (bytes == 2) to_global(static_cast<uint16_t*>(p))[i] = (uint16_t)v;
    else if (bytes == 4) to_global(static_cast<uint32_t*>(p))[i] = (uint32_t)v;
    else to_global(static_cast<uint64_t*>(p))[i] = v;
}

template <bool ORD>
__global__ __launch_bounds__(kWaveThreads) void k_seg_wave(SegCtx x) {
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t count = x.ctr[ctr_wave()];
    if (count == 0) return;  // empty bin: skip the shared counter
    for (;;) {
        uint32_t item = 0;
        if (lane == 0) item = atomicAdd(&x.ctr[ctr_wave_taken()], 1u);
        item = __builtin_amdgcn_readfirstlane(item);
        if (item >= count) break;
        const fs_segment d = x.segs[x.wave_list[item]];
        const uint32_t n = (uint32_t)d.n;
        const int kb = (int)d.key_bits / 8, vb = (int)d.val_bytes;
        const bool valid = lane < n;
        const uint64_t k = valid ? load_elem(d.keys_in, lane, kb) : 0;
        // the order-mapped key, as an unsigned value of the segment's width
        uint64_t t = k;
        if constexpr (ORD) {
            const int w = kb == 2 ? 0 : kb == 4 ? 1 : 2;
            const uint64_t top = k >> (8 * kb - 1);
            t = k ^ (top ? x.ord_neg[w] : x.ord_pos[w]);
            if (kb < 8) t &= (1ull << (8 * kb)) - 1;
        }
        uint32_t rank = 0;
        for (uint32_t j = 0; j < n; ++j) {
            const uint64_t tj = ((uint64_t)__shfl((int)(uint32_t)(t >> 32), (int)j, 64) << 32) |
                                (uint32_t)__shfl((int)(uint32_t)t, (int)j, 64);
            rank += (tj < t || (tj == t && j < lane)) ? 1u : 0u;
        }
        if (valid) {
            store_elem(d.keys_out, rank, kb, k);
            if (vb) store_elem(d.vals_out, rank, vb, load_elem(d.vals_in, lane, vb));
        }
    }
}

template <bool ORD>
__global__ __launch_bounds__(kSmallThreads) void k_seg_small(SegCtx x) {
    __shared__ SmallShared sm;
    const int tid = threadIdx.x;
    for (int i = tid; i < kSmallWaves * kRadix; i += kSmallThreads) (&sm.peers[0][0])[i] = 0;
    const uint32_t nsmall = x.ctr[0];
    if (nsmall == 0) return;  // empty bin: skip the shared counter
    // queue entries are popped one segment ahead so that the pop overlaps the work
    if (tid == 0) sm.next = add_agent(&x.ctr[1], 1u);
    for (;;) {
        __syncthreads();
        if (tid == 0) {
            sm.seg = sm.next;
            if (sm.seg < nsmall) sm.next = add_agent(&x.ctr[1], 1u);
        }
        __syncthreads();
        const uint32_t i = sm.seg;
        if (i >= nsmall) break;
        const fs_segment d = x.segs[x.small_list[i]];
        switch (seg_class(d.key_bits / 8, d.val_bytes)) {
        case 0: sort_small<uint16_t, NoVal, ORD>(x, d, sm); break;
        case 1: sort_small<uint16_t, uint32_t, ORD>(x, d, sm); break;
        case 2: sort_small<uint16_t, uint64_t, ORD>(x, d, sm); break;
        case 3: sort_small<uint32_t, NoVal, ORD>(x, d, sm); break;
        case 4: sort_small<uint32_t, uint32_t, ORD>(x, d, sm); break;
        case 5: sort_small<uint32_t, uint64_t, ORD>(x, d, sm); break;
        case 6: sort_small<uint64_t, NoVal, ORD>(x, d, sm); break;
        case 7: sort_small<uint64_t, uint32_t, ORD>(x, d, sm); break;
        default: sort_small<uint64_t, uint64_t, ORD>(x, d, sm); break;
        }
    }
}

// ---------------------------------------------------------------------------
// 16-bit-digit bin: 16-bit keys without payload.
//
// The whole key is one digit, so the histogram is the multiset of the
// segment and the sorted output is written straight from its prefix sums
// (Section III-E, with no index array).  The 2^16 counters are packed two per
// 32-bit LDS word (Section III-D.1), which is what lets the full histogram
// sit in one workgroup's LDS.  A count past 65535 needs the carry repair of
// the packed pair; carries are rare (one per 65536 keys of a bin) and are
// logged in LDS, with a bit per word that has any.
//
// Medium segments take one workgroup each.  Long segments are split into
// parts of kX16Part keys: one launch builds each part's histogram in LDS and
// adds its exact counts to the segment's global histogram (the local-then-
// global merge of Section III-A); a second launch gives each part of the
// OUTPUT a workgroup that loads the segment's counts back into the packed LDS
// form, takes their prefix sums and writes its share of the sorted keys.
// ---------------------------------------------------------------------------
constexpr int kExpThreads = 1024;
constexpr int kExpGroups = 4096;    // 16-bin groups of the 2^16 bins
constexpr int kExpEvents = 256;     // carry log (a segment below 2^23 keys logs fewer than 256)

struct ExpandShared {
    __attribute__((aligned(16))) uint32_t cnt[kHist16Words];  // bins 2w (low half) and 2w+1 (high half)
    uint32_t gpre[kExpGroups];            // exclusive prefix of every 16-bin group
    uint32_t carried[kHist16Words / 32];  // one bit per word that logged a carry
    uint32_t ev[kExpEvents];              // word | (1 << 31 for a carry out of the whole word)
    uint32_t big_lo[kExpEvents];          // exact counts of the carried pairs (exp_settle);
    uint32_t big_hi[kExpEvents];          //   such a pair's word then holds its index here
    __attribute__((aligned(8))) uint16_t marks[kExpThreads / kWave][256];  // per-wave output marks
    uint32_t wsum[kExpThreads / kWave];
    uint32_t nev, nbig;
    uint32_t item, next;                  // queue entries: current and prefetched
};

// exact count of bin v (after exp_settle)
__device__ __forceinline__ uint32_t exp_count(const ExpandShared& sm, uint32_t v) {
    const uint32_t w = v >> 1;
    const uint32_t word = sm.cnt[w];
    if (__builtin_expect(!((sm.carried[w >> 5] >> (w & 31)) & 1u), 1))
        return (v & 1u) ? (word >> 16) : (word & 0xFFFFu);
    return (v & 1u) ? sm.big_hi[word] : sm.big_lo[word];
}

// Decode every carried pair once from the carry log into the exact-count
// table and leave the table index in its word, so that a count is one
// lookup however often it is read.  With W the word, nlo and nword the
// pair's low-half and whole-word carries:
//   lo = (W & 0xFFFF) + 2^16 nlo,  S = W + 2^32 nword = lo + 2^16 hi.
// Every thread must call it, after the histogram is complete; a barrier
// must follow.
__device__ __forceinline__ void exp_settle(ExpandShared& sm, uint32_t* err) {
    const uint32_t nev = sm.nev < (uint32_t)kExpEvents ? sm.nev : (uint32_t)kExpEvents;
    if (threadIdx.x == 0 && sm.nev > (uint32_t)kExpEvents) atomicOr(err, 64u);
    for (uint32_t cw = threadIdx.x; cw < (uint32_t)kHist16Words / 32; cw += kExpThreads) {
        uint32_t bits = sm.carried[cw];
        while (bits) {
            const uint32_t w = 32 * cw + (uint32_t)__builtin_ctz(bits);
            bits &= bits - 1;
            uint32_t nlo = 0, nword = 0;
            for (uint32_t e = 0; e < nev; ++e) {
                const uint32_t r = sm.ev[e];
                if ((r & 0x7FFFFFFFu) == w) {
                    if (r >> 31) ++nword;
                    else ++nlo;
                }
            }
            const uint32_t word = sm.cnt[w];
            const uint64_t lo = (uint64_t)(word & 0xFFFFu) + ((uint64_t)nlo << 16);
            const uint64_t sum = (uint64_t)word + ((uint64_t)nword << 32);
            const uint32_t k = atomicAdd(&sm.nbig, 1u);
            if (k < (uint32_t)kExpEvents) {
                sm.big_lo[k] = (uint32_t)lo;
                sm.big_hi[k] = (uint32_t)((sum - lo) >> 16);
                sm.cnt[w] = k;
            } else {
                atomicOr(err, 64u);
            }
        }
    }
}

__device__ __forceinline__ void exp_log(ExpandShared& sm, uint32_t w, uint32_t nlo, uint32_t nword) {
    atomicOr(&sm.carried[w >> 5], 1u << (w & 31));
    const uint32_t e = atomicAdd(&sm.nev, nlo + nword);
    for (uint32_t k = 0; k < nword; ++k)
        if (e + k < (uint32_t)kExpEvents) sm.ev[e + k] = w | 0x80000000u;
    for (uint32_t k = 0; k < nlo; ++k)
        if (e + nword + k < (uint32_t)kExpEvents) sm.ev[e + nword + k] = w;
}

__device__ __forceinline__ void exp_add_logged(ExpandShared& sm, uint32_t key) {
    const uint32_t w = key >> 1;
    const uint32_t inc = (key & 1u) ? 0x10000u : 1u;
    const uint32_t old = atomicAdd(&sm.cnt[w], inc);
    const bool word_wrap = old + inc < old;
    const bool lo_wrap = (old & 0xFFFFu) + (inc & 0xFFFFu) > 0xFFFFu;
    if (__builtin_expect(word_wrap || lo_wrap, 0)) exp_log(sm, w, (uint32_t)lo_wrap, (uint32_t)word_wrap);
}

__device__ __forceinline__ void exp_clear(ExpandShared& sm) {
    const int tid = threadIdx.x;
    u32x4* c4 = reinterpret_cast<u32x4*>(sm.cnt);
    const u32x4 z = {0u, 0u, 0u, 0u};
    for (int i = tid; i < kHist16Words / 4; i += kExpThreads) c4[i] = z;
    for (int i = tid; i < kHist16Words / 32; i += kExpThreads) sm.carried[i] = 0;
    if (tid == 0) sm.nev = sm.nbig = 0;
}

// histogram of keys [0, n) of `keys`: aligned 16-byte loads, keys outside
// the range masked (an aligned 16-byte block never leaves a mapped page)
template <bool ORD>
__device__ __forceinline__ void exp_hist(const SegCtx& x, ExpandShared& sm, const uint16_t* keys, uint64_t n) {
    const int tid = threadIdx.x;
    const uintptr_t p = reinterpret_cast<uintptr_t>(keys);
    const uintptr_t a0 = p & ~(uintptr_t)15;
    const uint64_t lead = (p - a0) >> 1;
    const uint64_t nv = (lead + n + 7) >> 3;
    const gptr<const u32x4> vp = (gptr<const u32x4>)(a0);
    const bool may_carry = n > 0xFFFFu;  // no bin of a shorter range passes 65535
    constexpr int U = 4;                 // vectors in flight per thread
    for (uint64_t i0 = 0; i0 < nv; i0 += U * kExpThreads) {
        u32x4 v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint64_t i = i0 + (uint64_t)u * kExpThreads + tid;
            v[u] = __builtin_nontemporal_load(&vp[i < nv ? i : nv - 1]);
        }
        if constexpr (ORD) {
#pragma unroll
            for (int u = 0; u < U; ++u) v[u] = order_map_vec<uint16_t>(v[u], x.ord_pos[0], x.ord_neg[0]);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint64_t i = i0 + (uint64_t)u * kExpThreads + tid;
            const uint32_t wv[4] = {v[u].x, v[u].y, v[u].z, v[u].w};
            if (ballot(i * 8 >= lead && i * 8 + 8 <= lead + n) == ballot(true)) {
                // every lane's vector inside the range: an add of one per
                // key; a carry needs a half that read 0xFFFF, so only then
                // are the exact tests made
                uint32_t kk[8], sft[8], old[8];
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    kk[e] = (wv[e >> 1] >> (16 * (e & 1))) & 0xFFFFu;
                    sft[e] = (kk[e] & 1u) << 4;
                    old[e] = atomicAdd(&sm.cnt[kk[e] >> 1], 1u << sft[e]);
                }
                if (may_carry) {
                    bool full = false;
#pragma unroll
                    for (int e = 0; e < 8; ++e) full |= ((old[e] >> sft[e]) & 0xFFFFu) == 0xFFFFu;
                    if (__builtin_expect(full, 0)) {
#pragma unroll
                        for (int e = 0; e < 8; ++e) {
                            const uint32_t inc = 1u << sft[e];
                            const bool word_wrap = old[e] + inc < old[e];
                            const bool lo_wrap = (old[e] & 0xFFFFu) + (inc & 0xFFFFu) > 0xFFFFu;
                            if (word_wrap || lo_wrap) exp_log(sm, kk[e] >> 1, (uint32_t)lo_wrap, (uint32_t)word_wrap);
                        }
                    }
                }
                continue;
            }
            uint32_t w8[8], inc8[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const uint64_t idx = i * 8 + e;  // element index from a0; valid in [lead, lead + n)
                const bool valid = idx >= lead && idx < lead + n;
                const uint32_t key = (wv[e >> 1] >> (16 * (e & 1))) & 0xFFFFu;
                // a masked key adds 0 to a word picked by the lane (no conflict)
                w8[e] = valid ? key >> 1 : (threadIdx.x + 64u * e) & 0x7FFFu;
                inc8[e] = valid ? ((key & 1u) ? 0x10000u : 1u) : 0u;
            }
            if (may_carry) {
                // every returning add in flight before any carry is examined
                uint32_t old[8];
#pragma unroll
                for (int e = 0; e < 8; ++e) old[e] = atomicAdd(&sm.cnt[w8[e]], inc8[e]);
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    const bool word_wrap = old[e] + inc8[e] < old[e];
                    const bool lo_wrap = (old[e] & 0xFFFFu) + (inc8[e] & 0xFFFFu) > 0xFFFFu;
                    if (__builtin_expect(word_wrap || lo_wrap, 0))
                        exp_log(sm, w8[e], (uint32_t)lo_wrap, (uint32_t)word_wrap);
                }
            } else {
#pragma unroll
                for (int e = 0; e < 8; ++e)
                    if (inc8[e]) atomicAdd(&sm.cnt[w8[e]], inc8[e]);
            }
        }
    }
}

// exclusive prefix of the 16-bin groups (thread t owns groups 4t..4t+3)
__device__ __forceinline__ void exp_scan(ExpandShared& sm) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    uint32_t gs[4], tot = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int g = 4 * tid + k;
        uint32_t sum = 0;
        const u32x4* c4 = reinterpret_cast<const u32x4*>(&sm.cnt[8 * g]);
        const uint32_t flags = (sm.carried[(8 * g) >> 5] >> ((8 * g) & 31)) & 0xFFu;
        if (flags == 0) {
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const u32x4 q = c4[h];
                sum += (q.x & 0xFFFFu) + (q.x >> 16) + (q.y & 0xFFFFu) + (q.y >> 16) + (q.z & 0xFFFFu) +
                       (q.z >> 16) + (q.w & 0xFFFFu) + (q.w >> 16);
            }
        } else {
            for (int b = 0; b < 16; ++b) sum += exp_count(sm, 16u * g + b);
        }
        gs[k] = sum;
        tot += sum;
    }
    uint32_t inc = tot;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t y = __shfl_up(inc, off, 64);
        if (lane >= off) inc += y;
    }
    if (lane == 63) sm.wsum[wave] = inc;
    __syncthreads();
    uint32_t before = 0;
    for (int w = 0; w < wave; ++w) before += sm.wsum[w];
    uint32_t r = before + inc - tot;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        sm.gpre[4 * tid + k] = r;
        r += gs[k];
    }
}

// Write sorted positions [pa, pb) of the n-key output `out` from the LDS
// histogram.  Every wave takes an equal share of the positions (skewed
// histograms do not unbalance the waves) and finds the 16-bin group holding
// its first position once, by binary search over the group prefixes.  It
// then walks its share in chunks of 256 positions: one lane per group that
// starts in the chunk walks that group's 16 bins and marks, in the wave's
// LDS mark array, the chunk position where each non-empty bin starts (and
// the bin holding the chunk's first position); a wave max-scan fills every
// position with the last mark at or before it.  Every lane does the same
// work, so no lane's walk holds the others up.  Lane i writes positions
// 4i..4i+3 of the chunk with one aligned 8-byte store.
template <bool ORD>
__device__ __forceinline__ void exp_out(const SegCtx& x, const ExpandShared& sm, uint16_t* out, uint64_t n, uint64_t pa,
                                        uint64_t pb) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    constexpr int NW = kExpThreads / kWave;
    constexpr uint64_t kGroupCost = 8;  // a group walked costs about as much as 8 positions filled
    uint16_t* const marks = const_cast<uint16_t*>(sm.marks[wave]);
    // last group whose prefix is <= p, searched in [lo, kExpGroups)
    auto group_of = [&](uint64_t p, uint32_t lo) {
        uint32_t g = lo, len = (uint32_t)kExpGroups - lo;
        while (len > 1) {
            const uint32_t half = len >> 1;
            if (sm.gpre[g + half] <= p) g += half;
            len -= half;
        }
        return g;
    };
    // The wave's share of [pa, pb): cut points placed so that every wave
    // gets the same positions + kGroupCost * groups (a sparse key range costs
    // group walks, a dense one positions).  cost(g) is that measure at the
    // start of group g; inside a group it grows by one per position, so a
    // cut can fall inside a group and a hot group is shared by several waves.
    const uint32_t ga = group_of(pa, 0), gz = group_of(pb - 1, ga) + 1;
    auto pos_of = [&](uint32_t g) {
        const uint64_t p = g < (uint32_t)kExpGroups ? sm.gpre[g] : n;
        return p < pa ? pa : p > pb ? pb : p;
    };
    auto cost = [&](uint32_t g) { return pos_of(g) + kGroupCost * g; };
    const uint64_t c_lo = cost(ga), c_span = cost(gz) - c_lo;
    uint32_t g_w = ga;
    auto cut = [&](int w, uint32_t* gw) -> uint64_t {  // position of the w-th cut, and its group
        if (w == 0) {
            *gw = ga;
            return pa;
        }
        if (w == NW) {
            *gw = gz;
            return pb;
        }
        const uint64_t target = c_lo + c_span * (uint64_t)w / NW;
        uint32_t g = ga, len = gz - ga + 1;
        while (len > 1) {
            const uint32_t half = len >> 1;
            if (cost(g + half) <= target) g += half;
            len -= half;
        }
        *gw = g;
        const uint64_t p = pos_of(g) + (target - cost(g));
        const uint64_t pe = g < gz ? pos_of(g + 1) : pb;
        return p < pe ? p : pe;
    };
    uint32_t g_unused;
    const uint64_t A = cut(wave, &g_w), B = cut(wave + 1, &g_unused);
    if (A >= B) return;
    uint32_t gc = g_w;  // at or before the group holding A
    // 8-byte output quads: quad q holds positions 4q - lead .. 4q - lead + 3
    const uint32_t lead = (uint32_t)((reinterpret_cast<uintptr_t>(out) & 7) >> 1);
    for (uint64_t qc = (A + lead) >> 2;; qc += 64) {
        const int64_t c0 = (int64_t)(4 * qc) - (int64_t)lead;  // chunk position of mark 0
        if (c0 >= (int64_t)B) break;
        const uint64_t f = c0 > (int64_t)A ? (uint64_t)c0 : A;  // first position written
        const uint64_t cend = (uint64_t)(c0 + 256) < B ? (uint64_t)(c0 + 256) : B;
        reinterpret_cast<uint64_t*>(marks)[lane] = 0;
        __builtin_amdgcn_wave_barrier();
        // marks hold v - 16 gc (0 also for "no mark": the bin at f is the
        // smallest, so filling from it is right either way)
        const uint32_t vbase = 16u * gc;
        uint32_t glast = gc;
        for (uint32_t gb = gc;; gb += 64) {
            // the group holding f, and every group that starts inside the
            // chunk (not the empty groups whose prefix is the chunk's end)
            const uint32_t g = gb + lane;
            const bool act = g < (uint32_t)kExpGroups && (g == gc || sm.gpre[g] < cend);
            if (act) {
                uint32_t c[16];
                const uint32_t w0 = 8 * g;
                if ((sm.carried[w0 >> 5] >> (w0 & 31)) & 0xFFu) {
#pragma unroll
                    for (int b = 0; b < 16; ++b) c[b] = exp_count(sm, 16 * g + b);
                } else {
                    const u32x4* c4 = reinterpret_cast<const u32x4*>(&sm.cnt[w0]);
                    const u32x4 q0 = c4[0], q1 = c4[1];
                    const uint32_t wd[8] = {q0.x, q0.y, q0.z, q0.w, q1.x, q1.y, q1.z, q1.w};
#pragma unroll
                    for (int b = 0; b < 16; ++b) c[b] = (b & 1) ? wd[b >> 1] >> 16 : wd[b >> 1] & 0xFFFFu;
                }
                uint64_t st = sm.gpre[g];
#pragma unroll
                for (int b = 0; b < 16; ++b) {
                    const uint32_t v = 16 * g + b;
                    if (c[b]) {
                        if (st >= f && st < cend)
                            marks[st - c0] = (uint16_t)(v - vbase);  // a bin starting inside the chunk
                        else if (st < f && f < st + c[b])
                            marks[f - c0] = (uint16_t)(v - vbase);   // the bin holding the first position
                    }
                    st += c[b];
                }
            }
            const uint64_t am = ballot(act);
            if (am) glast = gb + 63 - (uint32_t)__builtin_clzll(am);
            if (am != ~0ull) break;  // group prefixes only grow: no later group starts in the chunk
        }
        __builtin_amdgcn_wave_barrier();
        // fill forward: inclusive max-scan over the 256 marks, 4 per lane
        const uint64_t m4 = reinterpret_cast<const uint64_t*>(marks)[lane];
        uint32_t r[4];
        r[0] = (uint32_t)(m4 & 0xFFFFu);
#pragma unroll
        for (int e = 1; e < 4; ++e) {
            const uint32_t me = (uint32_t)(m4 >> (16 * e)) & 0xFFFFu;
            r[e] = me > r[e - 1] ? me : r[e - 1];
        }
        uint32_t inc = r[3];
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const uint32_t y = __shfl_up(inc, off, 64);
            if (lane >= off && y > inc) inc = y;
        }
        uint32_t before = __shfl_up(inc, 1, 64);
        if (lane == 0) before = 0;
        uint32_t key[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) key[e] = seg_unmap<ORD, uint16_t>(x, (uint16_t)(vbase + (r[e] > before ? r[e] : before)));
        const int64_t p0 = c0 + 4 * lane;
        if (p0 >= (int64_t)f && (uint64_t)(p0 + 4) <= cend) {
            const uint64_t qv = (uint64_t)key[0] | ((uint64_t)key[1] << 16) | ((uint64_t)key[2] << 32) |
                                ((uint64_t)key[3] << 48);
            __builtin_nontemporal_store(qv, (gptr<uint64_t>)(reinterpret_cast<uintptr_t>(out + p0)));
        } else {
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int64_t pos = p0 + e;
                if (pos >= (int64_t)f && (uint64_t)pos < cend) to_global(out)[pos] = (uint16_t)key[e];
            }
        }
        __builtin_amdgcn_wave_barrier();
        gc = glast;  // at or before the group holding the next chunk's first position
    }
}

// medium segments: one workgroup per segment, queue entries popped one
// segment ahead so that the pop and the descriptor load overlap the work
template <bool ORD>
__global__ __launch_bounds__(kExpThreads) void k_seg_expand16(SegCtx x) {
    __shared__ ExpandShared sm;
    const int tid = threadIdx.x;
    const uint32_t nmed = x.ctr[ctr_expand_rest()];
    if (nmed == 0) return;  // empty bin: skip the shared counter
    uint32_t* taken = &x.ctr[ctr_expand_taken()];
    if (tid == 0) sm.next = add_agent(taken, 1u);
    for (;;) {
        __syncthreads();
        if (tid == 0) {
            sm.item = sm.next;
            if (sm.item < nmed) sm.next = add_agent(taken, 1u);
        }
        __syncthreads();
        const uint32_t i = sm.item;
        if (i >= nmed) break;
        const fs_segment d = x.segs[x.expand_list[x.nseg - 1 - i]];
        exp_clear(sm);
        __syncthreads();
        exp_hist<ORD>(x, sm, static_cast<const uint16_t*>(d.keys_in), d.n);
        __syncthreads();
        exp_settle(sm, x.err);
        __syncthreads();
        exp_scan(sm);
        __syncthreads();
        exp_out<ORD>(x, sm, static_cast<uint16_t*>(d.keys_out), d.n, 0, d.n);
    }
}

// ---- long segments (several workgroups each) --------------------------------

// part prefix over the long segments and the total part count (one block)
__global__ __launch_bounds__(1024) void k_seg_x16_layout(SegCtx x) {
    __shared__ uint32_t ws[16];
    const uint32_t cnt = x.ctr[ctr_expand_long()];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const uint32_t per = (cnt + 1023) / 1024;
    const uint32_t q0 = tid * per, q1 = q0 + per < cnt ? q0 + per : cnt;
    uint32_t lp = 0;
    for (uint32_t q = q0; q < q1; ++q) lp += (uint32_t)((x.segs[x.expand_list[q]].n + kX16Part - 1) / kX16Part);
    uint32_t ip = lp;
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t a = __shfl_up(ip, off, 64);
        if (lane >= off) ip += a;
    }
    if (lane == 63) ws[wave] = ip;
    __syncthreads();
    uint32_t before = 0, total = 0;
    for (int w = 0; w < 16; ++w) {
        if (w < wave) before += ws[w];
        total += ws[w];
    }
    uint32_t r = before + ip - lp;
    for (uint32_t q = q0; q < q1; ++q) {
        x.x16_parts[q] = r;
        r += (uint32_t)((x.segs[x.expand_list[q]].n + kX16Part - 1) / kX16Part);
    }
    if (tid == 0) {
        x.x16_parts[cnt] = total;
        x.ctr[ctr_x16_parts()] = total;
    }
}

__global__ void k_seg_x16_zero(SegCtx x) {
    const uint64_t words = (uint64_t)x.ctr[ctr_expand_long()] * 65536;
    u32x4* g4 = reinterpret_cast<u32x4*>(x.x16_hist);
    const u32x4 z = {0u, 0u, 0u, 0u};
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < words / 4;
         i += (uint64_t)gridDim.x * blockDim.x)
        g4[i] = z;
}

// the long segment holding part `part` (last q with x16_parts[q] <= part)
__device__ __forceinline__ uint32_t x16_segment_of(const SegCtx& x, uint32_t part, uint32_t nlong) {
    uint32_t q = 0, len = nlong;
    while (len > 1) {
        const uint32_t half = len >> 1;
        if (x.x16_parts[q + half] <= part) q += half;
        len -= half;
    }
    return q;
}

template <bool ORD>
__global__ __launch_bounds__(kExpThreads) void k_seg_x16_hist(SegCtx x) {
    __shared__ ExpandShared sm;
    const int tid = threadIdx.x;
    const uint32_t nlong = x.ctr[ctr_expand_long()];
    const uint32_t parts = x.ctr[ctr_x16_parts()];
    for (uint32_t part = blockIdx.x; part < parts; part += gridDim.x) {
        const uint32_t q = x16_segment_of(x, part, nlong);
        const fs_segment d = x.segs[x.expand_list[q]];
        const uint64_t b0 = (uint64_t)(part - x.x16_parts[q]) * kX16Part;
        const uint64_t m = d.n - b0 < kX16Part ? d.n - b0 : kX16Part;
        exp_clear(sm);
        __syncthreads();
        exp_hist<ORD>(x, sm, static_cast<const uint16_t*>(d.keys_in) + b0, m);
        __syncthreads();
        exp_settle(sm, x.err);
        __syncthreads();
        // add the exact nonzero counts to the segment's histogram
        uint32_t* gh = x.x16_hist + (uint64_t)q * 65536;
        for (uint32_t w = tid; w < (uint32_t)kHist16Words; w += kExpThreads) {
            const uint32_t word = sm.cnt[w];
            const bool carried = (sm.carried[w >> 5] >> (w & 31)) & 1u;
            const uint32_t lo = carried ? exp_count(sm, 2 * w) : word & 0xFFFFu;
            const uint32_t hi = carried ? exp_count(sm, 2 * w + 1) : word >> 16;
            if (lo) atomicAdd(&gh[2 * w], lo);
            if (hi) atomicAdd(&gh[2 * w + 1], hi);
        }
        __syncthreads();
    }
}

template <bool ORD>
__global__ __launch_bounds__(kExpThreads) void k_seg_x16_out(SegCtx x) {
    __shared__ ExpandShared sm;
    const int tid = threadIdx.x;
    const uint32_t nlong = x.ctr[ctr_expand_long()];
    const uint32_t parts = x.ctr[ctr_x16_parts()];
    for (uint32_t part = blockIdx.x; part < parts; part += gridDim.x) {
        const uint32_t q = x16_segment_of(x, part, nlong);
        const fs_segment d = x.segs[x.expand_list[q]];
        const uint64_t pa = (uint64_t)(part - x.x16_parts[q]) * kX16Part;
        const uint64_t pb = d.n - pa < kX16Part ? d.n : pa + kX16Part;
        // the segment's exact counts back into the packed LDS form; a pair
        // with a count past 65535 goes to the exact-count table
        if (tid < kHist16Words / 32) sm.carried[tid] = 0;
        if (tid == 0) sm.nbig = 0;
        __syncthreads();
        const uint32_t* gh = x.x16_hist + (uint64_t)q * 65536;
        for (uint32_t w = tid; w < (uint32_t)kHist16Words; w += kExpThreads) {
            const uint32_t lo = gh[2 * w], hi = gh[2 * w + 1];
            if (__builtin_expect((lo | hi) > 0xFFFFu, 0)) {
                const uint32_t k = atomicAdd(&sm.nbig, 1u);
                if (k < (uint32_t)kExpEvents) {
                    sm.big_lo[k] = lo;
                    sm.big_hi[k] = hi;
                    sm.cnt[w] = k;
                    atomicOr(&sm.carried[w >> 5], 1u << (w & 31));
                } else {
                    atomicOr(x.err, 64u);
                }
            } else {
                sm.cnt[w] = lo | (hi << 16);
            }
        }
        __syncthreads();
        exp_scan(sm);
        __syncthreads();
        exp_out<ORD>(x, sm, static_cast<uint16_t*>(d.keys_out), d.n, pa, pb);
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Large segments of one width class.
// ---------------------------------------------------------------------------
constexpr int kSegTileThreads = 256;

// tile and element prefixes over the class's large segments (one block)
__global__ __launch_bounds__(1024) void k_seg_layout(SegCtx x, int c) {
    __shared__ uint64_t wt[16], we[16];
    const uint32_t cnt = x.ctr[ctr_large(c)];
    const uint32_t* list = x.large_list + (uint64_t)c * x.nseg;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const uint32_t per = (cnt + 1023) / 1024;
    const uint32_t q0 = tid * per, q1 = q0 + per < cnt ? q0 + per : cnt;
    uint64_t lt = 0, le = 0;
    for (uint32_t q = q0; q < q1; ++q) {
        const uint64_t n = x.segs[list[q]].n;
        lt += (n + x.tile - 1) / x.tile;
        le += n;
    }
    uint64_t it = lt, ie = le;
    for (int off = 1; off < 64; off <<= 1) {
        const uint64_t a = __shfl_up(it, off, 64), b = __shfl_up(ie, off, 64);
        if (lane >= off) { it += a; ie += b; }
    }
    if (lane == 63) { wt[wave] = it; we[wave] = ie; }
    __syncthreads();
    uint64_t bt = 0, be = 0, tt = 0;
    for (int w = 0; w < 16; ++w) {
        if (w < wave) { bt += wt[w]; be += we[w]; }
        tt += wt[w];
    }
    uint64_t rt = bt + it - lt, re = be + ie - le;
    uint32_t* tp = x.tile_prefix;
    uint64_t* ep = x.elem_prefix;
    for (uint32_t q = q0; q < q1; ++q) {
        const uint64_t n = x.segs[list[q]].n;
        tp[q] = (uint32_t)rt;
        ep[q] = re;
        rt += (n + x.tile - 1) / x.tile;
        re += n;
    }
    if (tid == 0) {
        tp[cnt] = (uint32_t)tt;
        x.ctr[ctr_tiles(c)] = (uint32_t)tt;
    }
}

__global__ void k_seg_tilemap(SegCtx x, int c) {
    const uint32_t cnt = x.ctr[ctr_large(c)];
    for (uint32_t q = blockIdx.x * blockDim.x + threadIdx.x; q < cnt; q += gridDim.x * blockDim.x) {
        const uint32_t a = x.tile_prefix[q], b = x.tile_prefix[q + 1];
        for (uint32_t g = a; g < b && g < x.max_tiles; ++g) x.tile_seg[g] = q;
    }
}

// per-segment digit histograms: each workgroup takes a contiguous stretch
// of tiles and walks it one segment at a time, so the keys of a segment's
// tiles are read in one pipelined loop and the LDS counts are flushed once
// per segment.  Keys are read as aligned 16-byte vectors with the elements
// outside the range masked (an aligned 16-byte block never leaves a mapped
// page); when every valid lane of a wave has the same digit (long runs of one
// value, skewed keys) one lane adds the whole count.
template <typename K, bool ORD>
__global__ __launch_bounds__(kSegTileThreads) void k_seg_hist(SegCtx x, int c) {
    constexpr int D = sizeof(K);
    constexpr int VK = 16 / (int)sizeof(K);  // keys per vector
    constexpr int U = 4;                     // vectors in flight per thread
    __shared__ uint32_t cnt[D][kRadix];
    const uint32_t tiles = x.ctr[ctr_tiles(c)];
    const uint32_t* list = x.large_list + (uint64_t)c * x.nseg;
    const int tid = threadIdx.x;
    const uint32_t per = (tiles + gridDim.x - 1) / gridDim.x;
    const uint32_t g0 = blockIdx.x * per, g1 = g0 + per < tiles ? g0 + per : tiles;
    for (int i = tid; i < D * kRadix; i += kSegTileThreads) (&cnt[0][0])[i] = 0;
    __syncthreads();  // every counter is zero before any wave counts into it
    for (uint32_t g = g0; g < g1;) {
        const uint32_t q = x.tile_seg[g];
        const uint32_t tq0 = x.tile_prefix[q], tq1 = x.tile_prefix[q + 1];
        const uint32_t ge = tq1 < g1 ? tq1 : g1;  // this workgroup's tiles of segment q: [g, ge)
        const fs_segment d = x.segs[list[q]];
        const uint64_t b0 = (uint64_t)(g - tq0) * x.tile;
        const uint64_t b1 = (uint64_t)(ge - tq0) * x.tile < d.n ? (uint64_t)(ge - tq0) * x.tile : d.n;
        const uint64_t count = b1 - b0;
        const uintptr_t p = reinterpret_cast<uintptr_t>(static_cast<const K*>(d.keys_in) + b0);
        const uintptr_t a0 = p & ~(uintptr_t)15;
        const uint64_t lead = (p - a0) / sizeof(K);
        const uint64_t nv = (lead + count + VK - 1) / VK;
        const gptr<const u32x4> vp = (gptr<const u32x4>)(a0);
        for (uint64_t i0 = 0; i0 < nv; i0 += U * kSegTileThreads) {
            u32x4 v[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const uint64_t i = i0 + (uint64_t)u * kSegTileThreads + tid;
                v[u] = __builtin_nontemporal_load(&vp[i < nv ? i : nv - 1]);
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const uint64_t i = i0 + (uint64_t)u * kSegTileThreads + tid;
                const K* kv = reinterpret_cast<const K*>(&v[u]);
                const uint64_t all = ballot(true);
                if (ballot(i * VK >= lead && i * VK + VK <= lead + count) == all) {
                    // every lane's vector inside the range: a digit whose
                    // value differs across the wave's first keys (spread)
                    // adds one per key; the others keep the whole-wave test
                    uint32_t spread = 0;
                    const K k0 = seg_map<ORD, K>(x, kv[0]);
#pragma unroll
                    for (int j = 0; j < D; ++j) {
                        const uint32_t dg = digit_of<K>(k0, 8 * j);
                        if (ballot(dg == __builtin_amdgcn_readfirstlane(dg)) != all) spread |= 1u << j;
                    }
#pragma unroll
                    for (int e = 0; e < VK; ++e) {
                        const K key = seg_map<ORD, K>(x, kv[e]);
#pragma unroll
                        for (int j = 0; j < D; ++j) {
                            const uint32_t dg = digit_of<K>(key, 8 * j);
                            if ((spread >> j) & 1u) {
                                atomicAdd(&cnt[j][dg], 1u);
                            } else {
                                const uint32_t d0 = __builtin_amdgcn_readfirstlane(dg);
                                if (ballot(dg == d0) == all) {
                                    if (lanes_below(all) == 0) atomicAdd(&cnt[j][dg], popc64(all));
                                } else {
                                    atomicAdd(&cnt[j][dg], 1u);
                                }
                            }
                        }
                    }
                    continue;
                }
#pragma unroll
                for (int e = 0; e < VK; ++e) {
                    const uint64_t idx = i * VK + e;
                    const bool valid = idx >= lead && idx < lead + count;
                    const K key = seg_map<ORD, K>(x, kv[e]);
#pragma unroll
                    for (int j = 0; j < D; ++j) {
                        const uint32_t dg = digit_of<K>(key, 8 * j);
                        const uint32_t d0 = __builtin_amdgcn_readfirstlane(dg);
                        const uint64_t act = ballot(valid);
                        const uint64_t same = ballot(valid && dg == d0);
                        if (act != 0 && same == act) {
                            if (lanes_below(act) == 0 && valid) atomicAdd(&cnt[j][dg], popc64(act));
                        } else if (valid) {
                            atomicAdd(&cnt[j][dg], 1u);
                        }
                    }
                }
            }
        }
        __syncthreads();
        uint32_t* h = x.hist + (uint64_t)q * 8 * kRadix;
        for (int i = tid; i < D * kRadix; i += kSegTileThreads) {
            const uint32_t v = (&cnt[0][0])[i];
            if (v) atomicAdd(&h[i], v);
            (&cnt[0][0])[i] = 0;
        }
        __syncthreads();
        g = ge;
    }
}

// per segment: exclusive scan of every digit in place, trivial digits,
// pass plan (active, source, destination) and the copy flag
template <typename K>
__global__ __launch_bounds__(256) void k_seg_scan(SegCtx x, int c) {
    constexpr int D = sizeof(K);
    __shared__ uint64_t wsum[4];
    __shared__ uint32_t trivial[8];
    const uint32_t cnt = x.ctr[ctr_large(c)];
    const uint32_t* list = x.large_list + (uint64_t)c * x.nseg;
    const int b = threadIdx.x;
    for (uint32_t q = blockIdx.x; q < cnt; q += gridDim.x) {
        const uint64_t n = x.segs[list[q]].n;
        uint32_t* h = x.hist + (uint64_t)q * 8 * kRadix;
        for (int j = 0; j < D; ++j) {
            const uint32_t v = h[j * kRadix + b];
            uint64_t tot;
            const uint32_t e = (uint32_t)scan256_exclusive<uint64_t>(v, wsum, &tot);
            h[j * kRadix + b] = e;
            const int any = __syncthreads_or(v == n);
            if (b == 0) trivial[j] = any;
        }
        __syncthreads();
        if (b == 0) {
            int active = 0;
            for (int j = 0; j < D; ++j) active += trivial[j] ? 0 : 1;
            int i = 0;
            uint32_t prev = kBufIn;
            uint32_t* pl = x.plan + (uint64_t)q * 9;
            for (int j = 0; j < 8; ++j) {
                uint32_t w = 0;
                if (j < D && !trivial[j]) {
                    const uint32_t dst = ((active - 1 - i) % 2 == 0) ? kBufOut : kBufTmp;
                    w = 1u | (prev << 4) | (dst << 8);
                    prev = dst;
                    ++i;
                }
                pl[j] = w;
            }
            pl[8] = active == 0 ? 1u : 0u;
        }
        __syncthreads();
    }
}

// one stable scatter pass over digit j for all large segments of the class
// (tiles of THREADS * ITEMS keys; the tile layout used the same size).  The
// first 256 threads also own one digit value each for the tile's counts,
// its look-back and its output offsets.
template <typename K, typename V, int THREADS, int ITEMS, bool ORD>
__global__ __launch_bounds__(THREADS) void k_seg_scatter(SegCtx x, int c, int j) {
    constexpr int W = THREADS / kWave;
    constexpr int T = THREADS * ITEMS;
    constexpr bool kHasVals = !__is_same(V, NoVal);
    using VS = typename std::conditional<kHasVals, V, uint32_t>::type;
    __shared__ uint64_t s_peers[W][kRadix];
    __shared__ uint32_t s_wcnt[W][kRadix];
    __shared__ uint64_t s_delta[kRadix];
    __shared__ uint64_t s_wsum[4];
    __shared__ uint32_t s_ticket;
    __shared__ K s_keys[T];
    __shared__ VS s_vals[kHasVals ? T : 1];

    const uint32_t tiles = x.ctr[ctr_tiles(c)];
    // a class without large segments: leave before the ticket, whose one
    // counter every workgroup would otherwise hit at once
    if (tiles == 0) return;
    const uint32_t epoch = (uint32_t)(1 + 8 * c + j) << (kSegCountBits + 2);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int shift = 8 * j;
    for (int i = tid; i < W * kRadix; i += THREADS) (&s_peers[0][0])[i] = 0;
    uint32_t* ticket = &x.ctr[ctr_ticket(c, j)];
    const bool owner = tid < kRadix;  // owns digit value b = tid
    const int b = owner ? tid : 0;

    for (;;) {
        __syncthreads();
        if (tid == 0) s_ticket = add_agent(ticket, 1u);
        __syncthreads();
        const uint32_t g = __builtin_amdgcn_readfirstlane(s_ticket);
        if (g >= tiles) break;
        const SegTileDesc td = x.tdesc[g];  // one record: the segment and this pass's plan
        const uint32_t pl = ((j < 4 ? td.plan[0] : td.plan[1]) >> (8 * (j & 3))) & 0xFFu;
        if (!(pl & 1u)) continue;  // trivial digit of this segment
        const uint32_t q = td.q, t = td.t;
        const uint32_t src = (pl >> 1) & 3u, dstsel = (pl >> 3) & 3u;
        const uint64_t eo = td.eo;
        const auto src_k = to_global(src == kBufIn ? static_cast<const K*>(td.kin)
                                     : src == kBufOut ? static_cast<const K*>(td.kout)
                                                      : reinterpret_cast<const K*>(x.tmp_k) + eo);
        const auto dst_k = to_global(dstsel == kBufOut ? static_cast<K*>(td.kout)
                                                       : reinterpret_cast<K*>(x.tmp_k) + eo);
        gptr<const VS> src_v = nullptr;
        gptr<VS> dst_v = nullptr;
        if constexpr (kHasVals) {
            src_v = to_global(src == kBufIn ? static_cast<const VS*>(td.vin)
                              : src == kBufOut ? static_cast<const VS*>(td.vout)
                                               : reinterpret_cast<const VS*>(x.tmp_v) + eo);
            dst_v = to_global(dstsel == kBufOut ? static_cast<VS*>(td.vout)
                                                : reinterpret_cast<VS*>(x.tmp_v) + eo);
        }
        const uint64_t tb = (uint64_t)t * T;
        const uint32_t count = (uint32_t)((td.n - tb) < (uint64_t)T ? (td.n - tb) : (uint64_t)T);
        const uint32_t wbase = (uint32_t)wave * kWave * ITEMS;
        K key[ITEMS];
        VS val[ITEMS];
#pragma unroll
        for (int k = 0; k < ITEMS; ++k) {
            // every lane loads (clamped into the tile), so no load waits on a branch
            const uint32_t idx = wbase + k * kWave + lane;
            const uint32_t ic = idx < count ? idx : count - 1;
            key[k] = seg_map<ORD, K>(x, src_k[tb + ic]);
            if constexpr (kHasVals) val[k] = src_v[tb + ic];
        }
        for (int i = 0; i < kRadix / kWave; ++i) s_wcnt[wave][lane + kWave * i] = 0;
        __builtin_amdgcn_wave_barrier();
        uint32_t rank[ITEMS];
#pragma unroll
        for (int k = 0; k < ITEMS; ++k) {
            const bool valid = wbase + k * kWave + lane < count;
            rank[k] = wave_rank(digit_of<K>(key[k], shift), valid, s_peers[wave], s_wcnt[wave]);
        }
        __syncthreads();
        uint32_t h = 0;
        if (owner)
            for (int w = 0; w < W; ++w) h += s_wcnt[w][b];
        uint32_t* st = x.state + (uint64_t)g * kRadix;
        if (owner) st_agent(&st[b], epoch | (t == 0 ? kSegPrefix : kSegAgg) | h);
        uint64_t tot;
        const uint32_t start = (uint32_t)scan256_exclusive<uint64_t>(h, s_wsum, &tot);
        if (owner) {
            uint32_t r = start;
            for (int w = 0; w < W; ++w) {
                const uint32_t cc = s_wcnt[w][b];
                s_wcnt[w][b] = r;
                r += cc;
            }
        }
        uint32_t excl = 0;
        if (owner && t > 0) {
            int64_t p = (int64_t)g - 1;
            const int64_t first = (int64_t)g - t;  // tile 0 of this segment
            uint32_t spins = 0;
            for (;;) {
                uint32_t sw = ld_agent(&x.state[(uint64_t)p * kRadix + b]);
                if ((sw & ~((1u << (kSegCountBits + 2)) - 1)) != epoch || (sw & (kSegAgg | kSegPrefix)) == 0) {
                    if (++spins > kSpinLimit) {
                        atomicOr(x.err, 1u);
                        break;
                    }
                    __builtin_amdgcn_s_sleep(1);
                    continue;
                }
                excl += sw & kSegCountMask;
                if (sw & kSegPrefix) break;
                if (--p < first) {
                    atomicOr(x.err, 2u);
                    break;
                }
            }
            st_agent(&st[b], epoch | kSegPrefix | (excl + h));
        }
        if (owner) {
            const uint64_t gb = (uint64_t)x.hist[(uint64_t)q * 8 * kRadix + j * kRadix + b] + excl;
            s_delta[b] = gb - start;
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < ITEMS; ++k) {
            if (wbase + k * kWave + lane < count) {
                const uint32_t pos = s_wcnt[wave][digit_of<K>(key[k], shift)] + rank[k];
                if (pos < (uint32_t)T) {
                    s_keys[pos] = key[k];
                    if constexpr (kHasVals) s_vals[pos] = val[k];
                } else {
                    atomicOr(x.err, 4u);
                }
            }
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < ITEMS; ++k) {
            const uint32_t qq = k * THREADS + tid;
            if (qq < count) {
                const K kk = s_keys[qq];
                const uint64_t o = s_delta[digit_of<K>(kk, shift)] + qq;
                if (o < td.n) {
                    dst_k[o] = seg_unmap<ORD, K>(x, kk);
                    if constexpr (kHasVals) dst_v[o] = s_vals[qq];
                } else {
                    atomicOr(x.err, 8u);
                }
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Large segments of at most wg_max keys: one workgroup per segment, passes
// through global memory.  The workgroup owns the whole segment, so a pass
// walks the tiles in input order and carries each digit value's next output
// position from tile to tile in LDS: the stable scatter needs no look-back
// and no workgroup waits for another.
// ---------------------------------------------------------------------------
template <typename K, typename V, int ITEMS, bool ORD>
__global__ __launch_bounds__(256) void k_seg_wg(SegCtx x, int c) {
    constexpr int THREADS = 256;
    constexpr int W = THREADS / kWave;
    constexpr int T = THREADS * ITEMS;
    constexpr int D = sizeof(K);
    constexpr int VK = 16 / (int)sizeof(K);
    constexpr bool kHasVals = !__is_same(V, NoVal);
    using VS = typename std::conditional<kHasVals, V, uint32_t>::type;
    __shared__ uint64_t s_peers[W][kRadix];
    __shared__ uint32_t s_wcnt[W][kRadix];
    __shared__ uint32_t s_start[D][kRadix];  // digit histograms, then their exclusive prefixes
    __shared__ uint32_t s_next[kRadix];      // next output position of each digit value in this pass
    __shared__ uint32_t s_delta[kRadix];     // output position minus staged position, this tile
    __shared__ uint64_t s_wsum[4];
    __shared__ uint32_t s_trivial[D];
    __shared__ uint32_t s_item, s_next_item;
    __shared__ unsigned long long s_eo;
    __shared__ K s_keys[T];
    __shared__ VS s_vals[kHasVals ? T : 1];

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const uint32_t cnt = x.ctr[ctr_wg(c)];
    if (cnt == 0) return;  // no segment of this class: skip the shared counter
    const uint32_t* list = x.wg_list + (uint64_t)c * x.nseg;
    uint32_t* taken = &x.ctr[ctr_wg_taken(c)];
    for (int i = tid; i < W * kRadix; i += THREADS) (&s_peers[0][0])[i] = 0;
    if (tid == 0) s_next_item = add_agent(taken, 1u);
    for (;;) {
        __syncthreads();
        if (tid == 0) {
            s_item = s_next_item;
            if (s_item < cnt) s_next_item = add_agent(taken, 1u);
        }
        __syncthreads();
        const uint32_t item = s_item;
        if (item >= cnt) break;
        const fs_segment d = x.segs[list[item]];
        const uint32_t n = (uint32_t)d.n;
        if (tid == 0)
            s_eo = atomicAdd(reinterpret_cast<unsigned long long*>(&x.ctr[ctr_wg_tmp(c)]), (unsigned long long)n);
        for (int i = tid; i < D * kRadix; i += THREADS) (&s_start[0][0])[i] = 0;
        __syncthreads();
        // 1. every digit's histogram in one read (aligned 16-byte vectors,
        //    elements outside the segment masked; wave-uniform digits added once)
        {
            const uintptr_t p = reinterpret_cast<uintptr_t>(d.keys_in);
            const uintptr_t a0 = p & ~(uintptr_t)15;
            const uint32_t lead = (uint32_t)((p - a0) / sizeof(K));
            const uint32_t nv = (lead + n + VK - 1) / VK;
            const gptr<const u32x4> vp = (gptr<const u32x4>)(a0);
            constexpr int U = 4;
            for (uint32_t i0 = 0; i0 < nv; i0 += U * THREADS) {
                u32x4 v[U];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const uint32_t i = i0 + u * THREADS + tid;
                    v[u] = __builtin_nontemporal_load(&vp[i < nv ? i : nv - 1]);
                }
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const uint32_t i = i0 + u * THREADS + tid;
                    const K* kv = reinterpret_cast<const K*>(&v[u]);
                    const uint64_t all = ballot(true);
                    if (ballot(i < nv && i * VK >= lead && i * VK + VK <= lead + n) == all) {
                        // whole vectors: digits that differ across the wave's
                        // first keys add one per key (as in k_seg_hist)
                        uint32_t spread = 0;
                        const K k0 = seg_map<ORD, K>(x, kv[0]);
#pragma unroll
                        for (int j = 0; j < D; ++j) {
                            const uint32_t dg = digit_of<K>(k0, 8 * j);
                            if (ballot(dg == __builtin_amdgcn_readfirstlane(dg)) != all) spread |= 1u << j;
                        }
#pragma unroll
                        for (int e = 0; e < VK; ++e) {
                            const K ke = seg_map<ORD, K>(x, kv[e]);
#pragma unroll
                            for (int j = 0; j < D; ++j) {
                                const uint32_t dg = digit_of<K>(ke, 8 * j);
                                if ((spread >> j) & 1u) {
                                    atomicAdd(&s_start[j][dg], 1u);
                                } else if (ballot(dg == __builtin_amdgcn_readfirstlane(dg)) == all) {
                                    if (lanes_below(all) == 0) atomicAdd(&s_start[j][dg], popc64(all));
                                } else {
                                    atomicAdd(&s_start[j][dg], 1u);
                                }
                            }
                        }
                        continue;
                    }
#pragma unroll
                    for (int e = 0; e < VK; ++e) {
                        const uint32_t idx = i * VK + e;
                        const bool valid = i < nv && idx >= lead && idx < lead + n;
                        const K ke = seg_map<ORD, K>(x, kv[e]);
#pragma unroll
                        for (int j = 0; j < D; ++j) {
                            const uint32_t dg = digit_of<K>(ke, 8 * j);
                            const uint32_t d0 = __builtin_amdgcn_readfirstlane(dg);
                            const uint64_t act = ballot(valid);
                            if (act != 0 && ballot(valid && dg == d0) == act) {
                                if (lanes_below(act) == 0 && valid) atomicAdd(&s_start[j][dg], popc64(act));
                            } else if (valid) {
                                atomicAdd(&s_start[j][dg], 1u);
                            }
                        }
                    }
                }
            }
        }
        __syncthreads();
        // 2. exclusive prefix of every digit; trivial digits
        for (int j = 0; j < D; ++j) {
            const uint32_t h = s_start[j][tid];
            uint64_t tot;
            const uint32_t e = (uint32_t)scan256_exclusive<uint64_t>(h, s_wsum, &tot);
            s_start[j][tid] = e;
            const int triv = __syncthreads_or(h == n);
            if (tid == 0) s_trivial[j] = triv;
        }
        __syncthreads();
        int active = 0;
        for (int j = 0; j < D; ++j) active += s_trivial[j] ? 0 : 1;
        if (active == 0) {  // already sorted: the output is the input
            for (uint32_t i = tid; i < n; i += THREADS) {
                to_global(static_cast<K*>(d.keys_out))[i] = to_global(static_cast<const K*>(d.keys_in))[i];
                if constexpr (kHasVals)
                    to_global(static_cast<VS*>(d.vals_out))[i] = to_global(static_cast<const VS*>(d.vals_in))[i];
            }
            continue;
        }
        // 3. the passes, ping-ponging so that the last one writes the output
        const uint64_t eo = s_eo;
        const K* src_k = static_cast<const K*>(d.keys_in);
        const VS* src_v = kHasVals ? static_cast<const VS*>(d.vals_in) : nullptr;
        int done = 0;
        for (int j = 0; j < D; ++j) {
            if (s_trivial[j]) continue;
            const bool to_out = (active - 1 - done) % 2 == 0;
            K* dst_k = to_out ? static_cast<K*>(d.keys_out) : reinterpret_cast<K*>(x.tmp_k) + eo;
            VS* dst_v = nullptr;
            if constexpr (kHasVals) dst_v = to_out ? static_cast<VS*>(d.vals_out) : reinterpret_cast<VS*>(x.tmp_v) + eo;
            const int shift = 8 * j;
            s_next[tid] = s_start[j][tid];
            for (uint32_t tb = 0; tb < n; tb += T) {
                const uint32_t count = n - tb < (uint32_t)T ? n - tb : (uint32_t)T;
                const uint32_t wbase = (uint32_t)wave * kWave * ITEMS;
                K key[ITEMS];
                VS val[ITEMS];
#pragma unroll
                for (int k = 0; k < ITEMS; ++k) {
                    const uint32_t idx = wbase + k * kWave + lane;
                    const uint32_t ic = idx < count ? idx : count - 1;
                    key[k] = seg_map<ORD, K>(x, to_global(src_k)[tb + ic]);
                    if constexpr (kHasVals) val[k] = to_global(src_v)[tb + ic];
                }
                for (int i = 0; i < kRadix / kWave; ++i) s_wcnt[wave][lane + kWave * i] = 0;
                __builtin_amdgcn_wave_barrier();
                uint32_t rank[ITEMS];
#pragma unroll
                for (int k = 0; k < ITEMS; ++k) {
                    const bool valid = wbase + k * kWave + lane < count;
                    rank[k] = wave_rank(digit_of<K>(key[k], shift), valid, s_peers[wave], s_wcnt[wave]);
                }
                __syncthreads();
                uint32_t h = 0;
                for (int w = 0; w < W; ++w) h += s_wcnt[w][tid];
                uint64_t tot;
                const uint32_t start = (uint32_t)scan256_exclusive<uint64_t>(h, s_wsum, &tot);
                {
                    uint32_t r = start;
                    for (int w = 0; w < W; ++w) {
                        const uint32_t cc = s_wcnt[w][tid];
                        s_wcnt[w][tid] = r;
                        r += cc;
                    }
                }
                s_delta[tid] = s_next[tid] - start;  // modulo 2^32; positions stay below n
                s_next[tid] += h;
                __syncthreads();
#pragma unroll
                for (int k = 0; k < ITEMS; ++k) {
                    if (wbase + k * kWave + lane < count) {
                        const uint32_t pos = s_wcnt[wave][digit_of<K>(key[k], shift)] + rank[k];
                        if (pos < (uint32_t)T) {
                            s_keys[pos] = key[k];
                            if constexpr (kHasVals) s_vals[pos] = val[k];
                        } else {
                            atomicOr(x.err, 4u);
                        }
                    }
                }
                __syncthreads();
#pragma unroll
                for (int k = 0; k < ITEMS; ++k) {
                    const uint32_t qq = k * THREADS + tid;
                    if (qq < count) {
                        const K kk = s_keys[qq];
                        const uint32_t o = s_delta[digit_of<K>(kk, shift)] + qq;
                        if (o < n) {
                            to_global(dst_k)[o] = seg_unmap<ORD, K>(x, kk);
                            if constexpr (kHasVals) to_global(dst_v)[o] = s_vals[qq];
                        } else {
                            atomicOr(x.err, 8u);
                        }
                    }
                }
            }
            __syncthreads();  // this pass's stores are visible to the workgroup's next pass
            src_k = dst_k;
            if constexpr (kHasVals) src_v = dst_v;
            ++done;
        }
    }
}

// one record per tile of the class's large segments (after the plans)
__global__ void k_seg_tiledesc(SegCtx x, int c) {
    const uint32_t tiles = x.ctr[ctr_tiles(c)];
    const uint32_t* list = x.large_list + (uint64_t)c * x.nseg;
    for (uint32_t g = blockIdx.x * blockDim.x + threadIdx.x; g < tiles; g += gridDim.x * blockDim.x) {
        const uint32_t q = x.tile_seg[g];
        const fs_segment d = x.segs[list[q]];
        SegTileDesc r;
        r.kin = d.keys_in;
        r.kout = d.keys_out;
        r.vin = d.vals_in;
        r.vout = d.vals_out;
        r.n = d.n;
        r.eo = x.elem_prefix[q];
        r.q = q;
        r.t = g - x.tile_prefix[q];
        uint32_t pk[2] = {0u, 0u};
        for (int j = 0; j < 8; ++j) {
            const uint32_t w = x.plan[(uint64_t)q * 9 + j];
            const uint32_t b = (w & 1u) | (((w >> 4) & 3u) << 1) | (((w >> 8) & 3u) << 3);
            pk[j >> 2] |= b << (8 * (j & 3));
        }
        r.plan[0] = pk[0];
        r.plan[1] = pk[1];
        x.tdesc[g] = r;
    }
}

// segments whose every digit is trivial are already sorted: copy them
template <typename K, typename V>
__global__ __launch_bounds__(256) void k_seg_copy(SegCtx x, int c) {
    constexpr bool kHasVals = !__is_same(V, NoVal);
    const uint32_t tiles = x.ctr[ctr_tiles(c)];
    const uint32_t* list = x.large_list + (uint64_t)c * x.nseg;
    for (uint32_t g = blockIdx.x; g < tiles; g += gridDim.x) {
        const uint32_t q = x.tile_seg[g];
        if (!x.plan[(uint64_t)q * 9 + 8]) continue;
        const fs_segment d = x.segs[list[q]];
        const uint64_t tb = (uint64_t)(g - x.tile_prefix[q]) * x.tile;
        const uint64_t te = tb + x.tile < d.n ? tb + x.tile : d.n;
        const auto kin = to_global(static_cast<const K*>(d.keys_in));
        const auto kout = to_global(static_cast<K*>(d.keys_out));
        for (uint64_t i = tb + threadIdx.x; i < te; i += 256) {
            kout[i] = kin[i];
            if constexpr (kHasVals)
                to_global(static_cast<V*>(d.vals_out))[i] = to_global(static_cast<const V*>(d.vals_in))[i];
        }
    }
}

__global__ void k_seg_zero_hist(SegCtx x, int c) {
    const uint64_t words = (uint64_t)x.ctr[ctr_large(c)] * 8 * kRadix;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < words; i += (uint64_t)gridDim.x * blockDim.x)
        x.hist[i] = 0;
}

// ---------------------------------------------------------------------------
template <typename K, typename V, bool ORD>
static hipError_t run_class(const SegCtx& x, int c, int persistent, int threads, int items, hipStream_t s) {
    k_seg_zero_hist<<<1024, 256, 0, s>>>(x, c);
    k_seg_layout<<<1, 1024, 0, s>>>(x, c);
    k_seg_tilemap<<<256, 256, 0, s>>>(x, c);
    k_seg_hist<K, ORD><<<persistent, kSegTileThreads, 0, s>>>(x, c);
    k_seg_scan<K><<<persistent, 256, 0, s>>>(x, c);
    k_seg_tiledesc<<<256, 256, 0, s>>>(x, c);
    for (int j = 0; j < (int)sizeof(K); ++j) {
        if (threads == 256) {
            if (items == 8) k_seg_scatter<K, V, 256, 8, ORD><<<persistent, 256, 0, s>>>(x, c, j);
            else k_seg_scatter<K, V, 256, 16, ORD><<<persistent, 256, 0, s>>>(x, c, j);
        } else {
            if (items == 8) k_seg_scatter<K, V, 512, 8, ORD><<<persistent, 512, 0, s>>>(x, c, j);
            else k_seg_scatter<K, V, 512, 16, ORD><<<persistent, 512, 0, s>>>(x, c, j);
        }
    }
    k_seg_copy<K, V><<<persistent, 256, 0, s>>>(x, c);
    if (items == 8) k_seg_wg<K, V, 8, ORD><<<persistent, 256, 0, s>>>(x, c);
    else k_seg_wg<K, V, 16, ORD><<<persistent, 256, 0, s>>>(x, c);
    return hipGetLastError();
}

uint32_t seg_max_tiles(uint64_t total_keys, uint32_t nseg) {
    return (uint32_t)(total_keys / kSegMinTile + nseg + 1);
}

bool seg_tuning_valid(const fs_seg_tuning& t) {
    return (t.tile_items == 8 || t.tile_items == 16) && (t.tile_threads == 256 || t.tile_threads == 512) &&
           t.large_wgs_per_cu >= 1 && t.large_wgs_per_cu <= 8 &&
           t.small_wgs_per_cu >= 1 && t.small_wgs_per_cu <= 4 && t.expand16_wgs_per_cu >= 1 &&
           t.expand16_wgs_per_cu <= 2;
}

// every launch after the classification, in the key-order instantiation ORD
template <bool ORD>
static hipError_t launch_bins(const SegCtx& x, const fs_seg_tuning& t, int cus, hipStream_t s) {
    const int xg = cus * (int)t.expand16_wgs_per_cu;
    k_seg_x16_layout<<<1, 1024, 0, s>>>(x);
    k_seg_x16_zero<<<1024, 256, 0, s>>>(x);
    k_seg_x16_hist<ORD><<<xg, kExpThreads, 0, s>>>(x);
    k_seg_x16_out<ORD><<<xg, kExpThreads, 0, s>>>(x);
    k_seg_expand16<ORD><<<xg, kExpThreads, 0, s>>>(x);
    k_seg_wave<ORD><<<cus * 2, kWaveThreads, 0, s>>>(x);
    k_seg_small<ORD><<<cus * (int)t.small_wgs_per_cu, kSmallThreads, 0, s>>>(x);
    const int P = cus * (int)t.large_wgs_per_cu;
    const int it = (int)t.tile_items, th = (int)t.tile_threads;
    hipError_t e;
    if ((e = run_class<uint16_t, NoVal, ORD>(x, 0, P, th, it, s)) != hipSuccess) return e;
    if ((e = run_class<uint16_t, uint32_t, ORD>(x, 1, P, th, it, s)) != hipSuccess) return e;
    if ((e = run_class<uint16_t, uint64_t, ORD>(x, 2, P, th, it, s)) != hipSuccess) return e;
    if ((e = run_class<uint32_t, NoVal, ORD>(x, 3, P, th, it, s)) != hipSuccess) return e;
    if ((e = run_class<uint32_t, uint32_t, ORD>(x, 4, P, th, it, s)) != hipSuccess) return e;
    if ((e = run_class<uint32_t, uint64_t, ORD>(x, 5, P, th, it, s)) != hipSuccess) return e;
    if ((e = run_class<uint64_t, NoVal, ORD>(x, 6, P, th, it, s)) != hipSuccess) return e;
    if ((e = run_class<uint64_t, uint32_t, ORD>(x, 7, P, th, it, s)) != hipSuccess) return e;
    return run_class<uint64_t, uint64_t, ORD>(x, 8, P, th, it, s);
}

hipError_t launch_segmented(const SegCtx& x0, const fs_seg_tuning& t, hipStream_t s) {
    const int cus = device_cu_count();
    SegCtx x = x0;
    x.tile = t.tile_threads * t.tile_items;
    for (int w = 0; w < 3; ++w) x.small_max[w] = t.small_max_keys[w] < kSegMinSmallMax ? kSegMinSmallMax : t.small_max_keys[w];
    x.expand_min = t.expand16_min_keys;
    x.split_min = t.expand16_split_keys < kX16MinSplit ? kX16MinSplit : t.expand16_split_keys;
    x.wg_max = t.large_wg_max_keys;
    k_seg_classify<<<(x.nseg + 255) / 256 < 1024 ? (x.nseg + 255) / 256 : 1024, 256, 0, s>>>(x);
    return x.ord ? launch_bins<true>(x, t, cus, s) : launch_bins<false>(x, t, cus, s);
}

}  // namespace fs
