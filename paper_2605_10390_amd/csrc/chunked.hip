// Two-pass stable sort of 16-bit keys with payloads, planned from per-chunk
// compressed 2^16-bin histograms (no inter-workgroup waiting at all).
//
// Paper: the sort is driven by a tree histogram of narrow counters built
// once per batch (Section III-A/B, Algorithm 1) and read back as prefix
// sums (GetIndex, Algorithm 3).  Here the input is cut into G chunks (the
// paper's batches, Section III-C) and each chunk gets its own 2^16-bin
// histogram (both 8-bit digits jointly, i.e. the whole tree of a 16-bit key)
// with packed 16-bit LDS counters, exactly repaired after wraps.  From the
// per-chunk trees every workgroup of both scatter passes learns, before it
// starts, where each of its digit runs goes:
//
//   pass 0 (low byte d0), workgroup c = chunk c:
//     O0[c][a] = P0[a] + sum_{c' < c} #{keys of chunk c' with d0 = a}
//   pass 1 (high byte d1): the pass-0 output is the sequence of runs
//     (a, c) (all keys of chunk c with d0 = a), a-major; workgroup w takes a
//     contiguous stretch of whole runs starting at run r_w = (a_w, c_w), and
//     O1[w][b] = P1[b] + sum_{a' < a_w} H[b][a'] + sum_{c' < c_w} J[c'][b][a_w]
//   where J[c][b][a] counts keys of chunk c with d1 = b and d0 = a, and
//   H = sum_c J is the global histogram.
//
// Each workgroup then streams its contiguous range tile by tile, keeping a
// running output position per digit in LDS (the paper's histogram reused
// from batch to batch, Section III-D), so its writes for one digit are
// contiguous across tiles and partially written cache lines are completed
// by the same compute unit, inside its own XCD's L2.
#include "fs_device.hpp"
#include "fs_internal.hpp"
#include "fs_plan.hpp"

namespace fs {

// ---------------------------------------------------------------------------
// chunk geometry shared by the histogram and pass-0 kernels
// ---------------------------------------------------------------------------
__host__ __device__ inline uint64_t chunk_span(uint64_t n, uint32_t chunks) {
    const uint64_t per = (n + chunks - 1) / chunks;
    return (per + 63) & ~63ull;
}
__host__ __device__ inline uint64_t chunk_lo(uint64_t n, uint32_t chunks, uint32_t c) {
    const uint64_t x = (uint64_t)c * chunk_span(n, chunks);
    return x < n ? x : n;
}

// ---------------------------------------------------------------------------
// Per-chunk compressed histogram of 16 key bits starting at `shift`.
// LDS word w packs bins 2w (low half) and 2w+1 (high half).  A returning LDS
// add shows the adding lane the old word, so it sees exactly when its add
// carried out of the low half or out of the word; it appends that event to
// the wrap log (chunk, word, kind).  The chunk's counters are flushed as
// plain 32-bit halves J[c][bin]; k_joint_fix then applies the log:
//   low-half carry:  J[c][2w] += 2^16 and J[c][2w+1] -= 1 (the carry landed there)
//   word carry:      J[c][2w+1] += 2^16
// which restores the exact counts (each half holds its count mod 2^16 plus
// the carries, and the log holds every lost multiple of 2^16).
// ---------------------------------------------------------------------------
struct WrapLog {
    uint32_t* count;
    uint32_t* entries;
    uint32_t capacity;
};

__device__ __forceinline__ void joint_add(uint32_t* cnt, uint32_t bin, uint32_t c, uint32_t chunk,
                                          const WrapLog& log) {
    const uint32_t w = bin >> 1;
    const uint32_t inc = (bin & 1u) ? (c << 16) : c;
    const uint32_t old = atomicAdd(&cnt[w], inc);
    const bool word_wrap = (old + inc) < old;
    const bool lo_wrap = ((old & 0xFFFFu) + (inc & 0xFFFFu)) > 0xFFFFu;
    if (__builtin_expect(word_wrap | lo_wrap, 0)) {
        // entry: chunk (16 bits) | word (15 bits) | kind (1 bit: 1 = word carry)
        if (lo_wrap) {
            const uint32_t i = atomicAdd(log.count, 1u);
            if (i < log.capacity) log.entries[i] = (chunk << 16) | (w << 1) | 0u;
        }
        if (word_wrap) {
            const uint32_t i = atomicAdd(log.count, 1u);
            if (i < log.capacity) log.entries[i] = (chunk << 16) | (w << 1) | 1u;
        }
    }
}

template <typename K>
__device__ __forceinline__ uint32_t bits16(K key, int shift) {
    return (uint32_t)((uint64_t)key >> shift) & 0xFFFFu;
}

template <typename K>
__global__ __launch_bounds__(kHist16Threads) void k_joint16(const K* __restrict__ keys, uint64_t n,
                                                            uint32_t chunks, int shift,
                                                            uint32_t* __restrict__ J, WrapLog log) {
    __shared__ uint32_t cnt[kHist16Words];
    const int tid = threadIdx.x;
    const uint32_t c = blockIdx.x;
    for (int i = tid; i < kHist16Words; i += kHist16Threads) cnt[i] = 0;
    __syncthreads();
    const uint64_t lo = chunk_lo(n, chunks, c), hi = chunk_lo(n, chunks, c + 1);
    constexpr int VK = 16 / sizeof(K);
    // scalar keys up to the first 16-byte boundary, vectors, scalar tail
    const uintptr_t addr = reinterpret_cast<uintptr_t>(keys + lo);
    uint64_t head = ((16 - (addr & 15)) & 15) / sizeof(K);
    if (head > hi - lo) head = hi - lo;
    const uint64_t nvec = (hi - lo - head) / VK;
    const uint64_t body = lo + head, tail = body + nvec * VK;
    const u32x4* vec = reinterpret_cast<const u32x4*>(keys + body);
    for (uint64_t v = tid; v < nvec; v += kHist16Threads) {
        const u32x4 q = __builtin_nontemporal_load(&vec[v]);
        K k[VK];
        __builtin_memcpy(k, &q, 16);
        uint32_t b[VK];
#pragma unroll
        for (int e = 0; e < VK; ++e) b[e] = bits16<K>(k[e], shift);
        // whole wave on one bin: one add for all of it
        bool same = true;
#pragma unroll
        for (int e = 1; e < VK; ++e) same &= b[e] == b[0];
        const uint32_t bw = __builtin_amdgcn_readfirstlane(b[0]);
        const uint64_t active = ballot(true);
        if (ballot(same && b[0] == bw) == active) {
            if (lanes_below(active) == 0) joint_add(cnt, bw, VK * popc64(active), c, log);
            continue;
        }
        // otherwise one add per run of equal bins within the lane
        uint32_t run = 1;
#pragma unroll
        for (int e = 0; e < VK - 1; ++e) {
            if (b[e + 1] == b[e]) {
                ++run;
            } else {
                joint_add(cnt, b[e], run, c, log);
                run = 1;
            }
        }
        joint_add(cnt, b[VK - 1], run, c, log);
    }
    for (uint64_t e = tid; e < head + (hi - tail); e += kHist16Threads) {
        const uint64_t i = e < head ? lo + e : tail + (e - head);
        joint_add(cnt, bits16<K>(keys[i], shift), 1u, c, log);
    }
    __syncthreads();
    // flush as unpacked 32-bit halves, bin order
    uint32_t* dst = J + (uint64_t)c * 65536;
    for (int w = tid; w < kHist16Words; w += kHist16Threads) {
        const uint32_t x = cnt[w];
        uint2 pair;
        pair.x = x & 0xFFFFu;
        pair.y = x >> 16;
        reinterpret_cast<uint2*>(dst)[w] = pair;
    }
}

__global__ void k_joint_fix(uint32_t* J, const uint32_t* log_count, const uint32_t* entries,
                            uint32_t capacity) {
    uint32_t m = *log_count;
    if (m > capacity) m = capacity;  // never reached: capacity bounds the wraps of n keys
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < m; i += gridDim.x * blockDim.x) {
        const uint32_t e = entries[i];
        const uint32_t c = e >> 16, w = (e >> 1) & 0x7FFFu;
        uint32_t* row = J + (uint64_t)c * 65536;
        if (e & 1u) {
            atomicAdd(&row[2 * w + 1], 0x10000u);
        } else {
            atomicAdd(&row[2 * w], 0x10000u);
            atomicAdd(&row[2 * w + 1], 0xFFFFFFFFu);  // -1: the carry it put there
        }
    }
}

// In place over chunks: J[c][k] <- sum_{c' < c} J[c'][k]  (column prefix);
// H[k] <- sum over all chunks.  One thread per bin.
__global__ __launch_bounds__(256) void k_joint_scan(uint32_t* J, uint32_t chunks, uint64_t* H) {
    const uint32_t k = blockIdx.x * 256 + threadIdx.x;
    uint64_t run = 0;
    for (uint32_t c = 0; c < chunks; ++c) {
        uint32_t* p = J + (uint64_t)c * 65536 + k;
        const uint32_t v = *p;
        *p = (uint32_t)run;  // < chunk-prefix of one bin; fits: chunk ranges < 2^32 keys each
        run += v;
    }
    H[k] = run;
}

// Global plan: digit histograms (d0 = low byte a, d1 = high byte b) as
// marginals of H, their exclusive scans P0/P1, trivial digits, the pass
// plan, and RP[b][a] = sum_{a' < a} H[b][a'].  One block of 256 threads.
__global__ __launch_bounds__(256) void k_plan16(const uint64_t* __restrict__ H, uint64_t n,
                                                uint64_t* hist, uint64_t* base, uint64_t* RP,
                                                uint32_t* plan) {
    const int t = threadIdx.x;
    uint64_t h[2] = {0, 0};
    uint64_t run = 0;
    for (int i = 0; i < 256; ++i) {
        h[0] += H[i * 256 + t];   // column t: d0 = t
        const uint64_t x = H[t * 256 + i];  // row t: d1 = t
        RP[t * 256 + i] = run;
        run += x;
    }
    h[1] = run;
    finish_plan(h, 2, n, hist, base, plan);
}

// Pass-0 offsets: O0[c][a] = P0[a] + sum_b Jprefix[c][b][a]; the extra row
// c = chunks is the end of every digit's block, P0[a] + H0[a].
__global__ __launch_bounds__(256) void k_offsets0(const uint32_t* __restrict__ Jp, uint32_t chunks,
                                                  const uint64_t* __restrict__ P0,
                                                  const uint64_t* __restrict__ H0, uint64_t* O0) {
    const uint32_t c = blockIdx.x, a = threadIdx.x;
    if (c == chunks) {
        O0[(uint64_t)c * 256 + a] = P0[a] + H0[a];
        return;
    }
    const uint32_t* row = Jp + (uint64_t)c * 65536;
    uint64_t s = 0;
    for (int b = 0; b < 256; ++b) s += row[b * 256 + a];
    O0[(uint64_t)c * 256 + a] = P0[a] + s;
}

// Pass-1 ranges: workgroup w starts at the first run r = a*G + c whose
// start O0[c][a] is >= w*n/W (runs are contiguous and ordered in the pass-0
// output).  start1[w] = that run's start (n past the end), run1[w] = r.
__global__ void k_bounds1(const uint64_t* __restrict__ O0, uint32_t chunks, uint64_t n, uint32_t W,
                          uint64_t* start1, uint32_t* run1) {
    const uint32_t w = blockIdx.x * blockDim.x + threadIdx.x;
    if (w > W) return;
    const uint32_t R = 256u * chunks;
    const uint64_t target = (w == W) ? n + 1 : (n * (uint64_t)w) / W;
    // first r in [0, R] with start(r) >= target (start(R) = n)
    uint32_t lo = 0, hi = R;
    while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        const uint64_t s = O0[(uint64_t)(mid % chunks) * 256 + mid / chunks];
        if (s >= target) hi = mid; else lo = mid + 1;
    }
    if (w == W) lo = R;
    run1[w] = lo;
    start1[w] = lo == R ? n : O0[(uint64_t)(lo % chunks) * 256 + lo / chunks];
}

// Pass-1 offsets: O1[w][b] = P1[b] + RP[b][a] + Jprefix[c][b][a] for the
// first run (a, c) of workgroup w.
__global__ __launch_bounds__(256) void k_offsets1(const uint32_t* __restrict__ Jp,
                                                  const uint64_t* __restrict__ RP,
                                                  const uint64_t* __restrict__ P1,
                                                  const uint64_t* __restrict__ H1, uint32_t chunks,
                                                  const uint32_t* __restrict__ run1, uint64_t* O1) {
    const uint32_t w = blockIdx.x, b = threadIdx.x;
    const uint32_t r = run1[w];
    uint64_t o;
    if (r >= 256u * chunks) {
        o = P1[b] + H1[b];
    } else {
        const uint32_t a = r / chunks, c = r % chunks;
        o = P1[b] + RP[b * 256 + a] + Jp[(uint64_t)c * 65536 + b * 256 + a];
    }
    O1[(uint64_t)w * 256 + b] = o;
}

// ---------------------------------------------------------------------------
// Range scatter: one workgroup per contiguous input range with known first
// output position of every digit value (offsets[g][d]).
//
// Per tile: the keys arrive with 16-byte loads into LDS (16-bit loads per
// lane cap the read rate far below the HBM rate), are read back in striped
// order (item k of lane l of wave w is tile slot w*64*ITEMS + k*64 + l, the
// input order), ranked per wave (each lane ORs its lane bit into an LDS word
// per digit, so the word read back is the set of lanes sharing its digit),
// staged in LDS in digit order and written as contiguous per-digit runs that
// continue where the previous tile of the same workgroup stopped.
// ---------------------------------------------------------------------------
template <typename V, int THREADS, int ITEMS>
__global__ __launch_bounds__(THREADS) void k_range_scatter16(RangeArgs a) {
    using K = uint16_t;
    constexpr int W = THREADS / kWave;
    constexpr int T = THREADS * ITEMS;
    constexpr int KV = 8;           // keys per 16-byte vector
    constexpr int NV = T / KV + 1;  // vectors covering any tile
    static_assert(NV <= 2 * THREADS, "two key vectors per thread cover a tile");
    static_assert(THREADS >= kRadix, "one thread per digit value");

    __shared__ uint64_t s_peers[W][kRadix];
    __shared__ uint32_t s_wcnt[W][kRadix];
    __shared__ uint64_t s_run[kRadix];    // next output position of each digit value
    __shared__ uint64_t s_delta[kRadix];  // output of tile slot q is s_delta[d] + q
    __shared__ uint64_t s_wsum[4];
    __shared__ __attribute__((aligned(16))) K s_keys[NV * KV];  // raw key vectors, then staged keys
    __shared__ V s_vals[T];

    if (!a.plan[4 * a.pass]) return;
    const uint32_t src_sel = a.plan[4 * a.pass + 1], dst_sel = a.plan[4 * a.pass + 2];
    const K* src_k = static_cast<const K*>(src_sel == kBufIn ? a.in_k : src_sel == kBufOut ? a.out_k : a.tmp_k);
    K* dst_k = static_cast<K*>(dst_sel == kBufOut ? a.out_k : a.tmp_k);
    const V* src_v = static_cast<const V*>(src_sel == kBufIn ? a.in_v : src_sel == kBufOut ? a.out_v : a.tmp_v);
    V* dst_v = static_cast<V*>(dst_sel == kBufOut ? a.out_v : a.tmp_v);

    const uint32_t g = blockIdx.x;
    uint64_t lo, hi;
    if (a.range_start) {
        lo = a.range_start[g];
        hi = a.range_start[g + 1];
    } else {
        lo = chunk_lo(a.n, a.ranges, g);
        hi = chunk_lo(a.n, a.ranges, g + 1);
    }
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const uint64_t lane_bit = 1ull << lane;
    for (int i = tid; i < W * kRadix; i += THREADS) (&s_peers[0][0])[i] = 0;
    if (tid < kRadix) s_run[tid] = a.offsets[(uint64_t)g * kRadix + tid];
    const uintptr_t kaddr = reinterpret_cast<uintptr_t>(src_k);
    const uint32_t wbase = (uint32_t)wave * kWave * ITEMS;

    // Software pipeline: the next tile's key vectors and payloads are loaded
    // into registers while the current tile is ranked, staged and written.
    u32x4 nkv[2];
    V nval[ITEMS];
    auto fetch = [&](uint64_t tb) {
        const uint32_t cnt = (uint32_t)((hi - tb) < (uint64_t)T ? (hi - tb) : T);
        const uintptr_t b0 = kaddr + 2 * tb, b1 = kaddr + 2 * (tb + cnt);
        const uintptr_t v0 = b0 & ~(uintptr_t)15;
        const uint32_t nv = (uint32_t)((((b1 + 15) & ~(uintptr_t)15) - v0) / 16);
        const u32x4* gv = reinterpret_cast<const u32x4*>(v0);
#pragma unroll
        for (int r = 0; r < 2; ++r) {
            const uint32_t v = tid + r * THREADS;
            if (v < nv) nkv[r] = __builtin_nontemporal_load(&gv[v]);
        }
#pragma unroll
        for (int k = 0; k < ITEMS; ++k) {
            const uint32_t idx = wbase + k * kWave + lane;
            if (idx < cnt) nval[k] = __builtin_nontemporal_load(&src_v[tb + idx]);
        }
    };
    if (lo < hi) fetch(lo);

    for (uint64_t tile_begin = lo; tile_begin < hi; tile_begin += T) {
        const uint32_t count = (uint32_t)((hi - tile_begin) < (uint64_t)T ? (hi - tile_begin) : T);
        // keys: every aligned 16-byte vector overlapping the tile (such a vector
        // lies inside a page the array occupies) was loaded; place it in LDS
        const uintptr_t b0 = kaddr + 2 * tile_begin, b1 = kaddr + 2 * (tile_begin + count);
        const uintptr_t v0 = b0 & ~(uintptr_t)15;
        const uint32_t nv = (uint32_t)((((b1 + 15) & ~(uintptr_t)15) - v0) / 16);
        const uint32_t sh = (uint32_t)(b0 - v0) / 2;  // tile key i sits at s_keys[i + sh]
#pragma unroll
        for (int r = 0; r < 2; ++r) {
            const uint32_t v = tid + r * THREADS;
            if (v < nv) reinterpret_cast<u32x4*>(s_keys)[v] = nkv[r];
        }
        V val[ITEMS];
#pragma unroll
        for (int k = 0; k < ITEMS; ++k) val[k] = nval[k];
#pragma unroll
        for (int i = 0; i < kRadix / kWave; ++i) s_wcnt[wave][lane + kWave * i] = 0;
        __syncthreads();
        if (tile_begin + T < hi) fetch(tile_begin + T);

        K key[ITEMS];
#pragma unroll
        for (int k = 0; k < ITEMS; ++k) {
            const uint32_t idx = wbase + k * kWave + lane;
            key[k] = idx < count ? s_keys[idx + sh] : (K)0;
        }
        uint32_t rank[ITEMS];
#pragma unroll
        for (int k = 0; k < ITEMS; ++k) {
            const bool valid = wbase + k * kWave + lane < count;
            const uint32_t d = digit_of<K>(key[k], a.shift);
            if (valid) atomicOr(&s_peers[wave][d], lane_bit);
            __builtin_amdgcn_wave_barrier();
            uint64_t peers = 0;
            uint32_t before = 0;
            if (valid) {
                peers = s_peers[wave][d];
                before = s_wcnt[wave][d];
            }
            __builtin_amdgcn_wave_barrier();
            const uint32_t below = lanes_below(peers);
            if (valid && below == 0) {
                s_peers[wave][d] = 0;
                s_wcnt[wave][d] = before + popc64(peers);
            }
            __builtin_amdgcn_wave_barrier();
            rank[k] = before + below;
        }
        __syncthreads();

        const int b = tid;
        uint32_t h = 0;
        if (b < kRadix) {
#pragma unroll
            for (int w = 0; w < W; ++w) h += s_wcnt[w][b];
        }
        uint64_t tile_total;
        const uint32_t start = (uint32_t)scan256_exclusive<uint64_t>(b < kRadix ? h : 0, s_wsum, &tile_total);
        if (b < kRadix) {
            uint32_t run = start;
#pragma unroll
            for (int w = 0; w < W; ++w) {
                const uint32_t c = s_wcnt[w][b];
                s_wcnt[w][b] = run;
                run += c;
            }
            const uint64_t r = s_run[b];
            s_delta[b] = r - start;
            s_run[b] = r + h;
        }
        __syncthreads();

#pragma unroll
        for (int k = 0; k < ITEMS; ++k) {
            if (wbase + k * kWave + lane < count) {
                const uint32_t pos = s_wcnt[wave][digit_of<K>(key[k], a.shift)] + rank[k];
                if (pos < (uint32_t)T) {
                    s_keys[pos] = key[k];
                    s_vals[pos] = val[k];
                } else {
                    atomicOr(a.err, 4u);
                }
            }
        }
        __syncthreads();

#pragma unroll
        for (int k = 0; k < ITEMS; ++k) {
            const uint32_t q = k * THREADS + tid;
            if (q < count) {
                const K kk = s_keys[q];
                const uint64_t dst = s_delta[digit_of<K>(kk, a.shift)] + q;
                if (dst < a.n) {
                    dst_k[dst] = kk;
                    dst_v[dst] = s_vals[q];
                } else {
                    atomicOr(a.err, 8u);
                }
            }
        }
        __syncthreads();
    }
}

#ifndef FS_RANGE_THREADS
#define FS_RANGE_THREADS 512
#endif
#ifndef FS_RANGE_ITEMS
#define FS_RANGE_ITEMS 8
#endif

int range_scatter16_per_cu(int val_bytes) {
    int per_cu = 0;
    const hipError_t e = val_bytes == 8
        ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_range_scatter16<uint64_t, FS_RANGE_THREADS, FS_RANGE_ITEMS>, FS_RANGE_THREADS, 0)
        : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_range_scatter16<uint32_t, FS_RANGE_THREADS, FS_RANGE_ITEMS>, FS_RANGE_THREADS, 0);
    return (e == hipSuccess && per_cu > 0) ? per_cu : 1;
}

hipError_t launch_range_scatter16(const RangeArgs& a, uint32_t groups, int val_bytes, hipStream_t s) {
    if (groups == 0) return hipSuccess;
    switch (val_bytes) {
    case 4: k_range_scatter16<uint32_t, FS_RANGE_THREADS, FS_RANGE_ITEMS><<<groups, FS_RANGE_THREADS, 0, s>>>(a); break;
    case 8: k_range_scatter16<uint64_t, FS_RANGE_THREADS, FS_RANGE_ITEMS><<<groups, FS_RANGE_THREADS, 0, s>>>(a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

uint64_t chunk_begin(uint64_t n, uint32_t chunks, uint32_t c) { return chunk_lo(n, chunks, c); }

hipError_t launch_joint16(const void* keys, uint64_t n, int key_bytes, int shift, uint32_t chunks,
                          uint32_t* J, uint32_t* log_count, uint32_t* log_entries, uint32_t capacity,
                          hipStream_t s) {
    WrapLog log{log_count, log_entries, capacity};
    switch (key_bytes) {
    case 2: k_joint16<uint16_t><<<chunks, kHist16Threads, 0, s>>>((const uint16_t*)keys, n, chunks, shift, J, log); break;
    case 4: k_joint16<uint32_t><<<chunks, kHist16Threads, 0, s>>>((const uint32_t*)keys, n, chunks, shift, J, log); break;
    default: k_joint16<uint64_t><<<chunks, kHist16Threads, 0, s>>>((const uint64_t*)keys, n, chunks, shift, J, log); break;
    }
    return hipGetLastError();
}

hipError_t launch_plan_chunked16(const Plan16& p, uint64_t n, hipStream_t s) {
    k_joint_fix<<<64, 256, 0, s>>>(p.J, p.log_count, p.log_entries, p.log_capacity);
    k_joint_scan<<<256, 256, 0, s>>>(p.J, p.chunks, p.H);
    k_plan16<<<1, 256, 0, s>>>(p.H, n, p.hist, p.base, p.RP, p.plan);
    // pass 0: chunk offsets from digit 0's prefix (base row 0)
    k_offsets0<<<p.chunks + 1, 256, 0, s>>>(p.J, p.chunks, p.base, p.hist, p.O0);
    k_bounds1<<<(p.ranges1 + 1 + 255) / 256, 256, 0, s>>>(p.O0, p.chunks, n, p.ranges1, p.start1, p.run1);
    k_offsets1<<<p.ranges1 + 1, 256, 0, s>>>(p.J, p.RP, p.base + 2 * kRadix, p.hist + kRadix, p.chunks,
                                          p.run1, p.O1);
    return hipGetLastError();
}

}  // namespace fs
