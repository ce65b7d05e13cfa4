// Batched segmented sort: many independent segments in one call.
//
// The paper processes its input as batches that each update the histogram
// and are handled serially or in parallel (Sections III-C, IV-D); here a
// batch is a caller segment and every segment gets exactly the result a
// stand-alone sort would give it.  Segment descriptors live in device
// memory, so the whole schedule is decided on the device:
//   1. classify: each segment goes to the small queue (it fits in one
//      workgroup's LDS) or to the large queue of its (key, value) width class;
//   2. small segments: persistent workgroups pop the queue and sort each
//      segment entirely in LDS (one read and one write of HBM);
//   3. large segments, per width class: tile layout, per-segment digit
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
// and one ticket per (class, pass)
__host__ __device__ inline int ctr_large(int c) { return 2 + c; }
__host__ __device__ inline int ctr_tiles(int c) { return 16 + c; }
__host__ __device__ inline int ctr_ticket(int c, int j) { return 32 + 8 * c + j; }
__host__ __device__ inline int ctr_seen() { return 119; }  // 64-bit running total of queued keys (8-byte aligned)

// ---------------------------------------------------------------------------
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
        if (d.n <= small_cap(kb, vb)) {
            const uint32_t i = atomicAdd(&x.ctr[0], 1u);
            x.small_list[i] = s;
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
    uint32_t seg;
};

template <typename K, typename V>
__device__ void sort_small(const fs_segment& d, SmallShared& sm) {
    constexpr bool kHasVals = !__is_same(V, NoVal);
    using VS = typename std::conditional<kHasVals, V, uint32_t>::type;
    constexpr int D = sizeof(K);
    constexpr int kb = sizeof(K), vb = kHasVals ? sizeof(VS) : 0;
    const uint32_t n = (uint32_t)d.n;
    const uint32_t cap = small_cap(kb, vb);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    K* kbuf[2] = {reinterpret_cast<K*>(sm.buf[0]), reinterpret_cast<K*>(sm.buf[1])};
    VS* vbuf[2] = {reinterpret_cast<VS*>(sm.buf[0] + small_val_offset(cap, kb)),
                   reinterpret_cast<VS*>(sm.buf[1] + small_val_offset(cap, kb))};
    const K* kin = static_cast<const K*>(d.keys_in);
    for (uint32_t i = tid; i < n; i += kSmallThreads) {
        kbuf[0][i] = kin[i];
        if constexpr (kHasVals) vbuf[0][i] = static_cast<const VS*>(d.vals_in)[i];
    }
    __syncthreads();
    int cur = 0;
    for (int j = 0; j < D; ++j) {
        const int shift = 8 * j;
        if (tid < kRadix) sm.hist[tid] = 0;
        __syncthreads();
        for (uint32_t i = tid; i < n; i += kSmallThreads) atomicAdd(&sm.hist[digit_of<K>(kbuf[cur][i], shift)], 1u);
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
                key[k] = valid ? kbuf[cur][base + idx] : (K)0;
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
                        kbuf[1 - cur][pos] = key[k];
                        if constexpr (kHasVals) vbuf[1 - cur][pos] = vbuf[cur][base + idx];
                    }
                }
            }
            __syncthreads();
        }
        cur = 1 - cur;
    }
    K* kout = static_cast<K*>(d.keys_out);
    for (uint32_t i = tid; i < n; i += kSmallThreads) {
        kout[i] = kbuf[cur][i];
        if constexpr (kHasVals) static_cast<VS*>(d.vals_out)[i] = vbuf[cur][i];
    }
    __syncthreads();
}

__global__ __launch_bounds__(kSmallThreads) void k_seg_small(SegCtx x) {
    __shared__ SmallShared sm;
    const int tid = threadIdx.x;
    for (int i = tid; i < kSmallWaves * kRadix; i += kSmallThreads) (&sm.peers[0][0])[i] = 0;
    const uint32_t nsmall = x.ctr[0];
    for (;;) {
        __syncthreads();
        if (tid == 0) sm.seg = add_agent(&x.ctr[1], 1u);
        __syncthreads();
        const uint32_t i = sm.seg;
        if (i >= nsmall) break;
        const fs_segment d = x.segs[x.small_list[i]];
        switch (seg_class(d.key_bits / 8, d.val_bytes)) {
        case 0: sort_small<uint16_t, NoVal>(d, sm); break;
        case 1: sort_small<uint16_t, uint32_t>(d, sm); break;
        case 2: sort_small<uint16_t, uint64_t>(d, sm); break;
        case 3: sort_small<uint32_t, NoVal>(d, sm); break;
        case 4: sort_small<uint32_t, uint32_t>(d, sm); break;
        case 5: sort_small<uint32_t, uint64_t>(d, sm); break;
        case 6: sort_small<uint64_t, NoVal>(d, sm); break;
        case 7: sort_small<uint64_t, uint32_t>(d, sm); break;
        default: sort_small<uint64_t, uint64_t>(d, sm); break;
        }
    }
}

// ---------------------------------------------------------------------------
// Large segments of one width class.
// ---------------------------------------------------------------------------
constexpr int kSegTileThreads = 256;
constexpr int kSegTileItems = 16;
constexpr uint32_t kSegTile = kSegTileThreads * kSegTileItems;

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
        lt += (n + kSegTile - 1) / kSegTile;
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
        rt += (n + kSegTile - 1) / kSegTile;
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

// per-segment digit histograms: each workgroup walks a contiguous stretch of
// tiles and flushes its LDS counts whenever the segment changes
template <typename K>
__global__ __launch_bounds__(kSegTileThreads) void k_seg_hist(SegCtx x, int c) {
    constexpr int D = sizeof(K);
    __shared__ uint32_t cnt[D][kRadix];
    __shared__ uint32_t s_q;
    const uint32_t tiles = x.ctr[ctr_tiles(c)];
    const uint32_t* list = x.large_list + (uint64_t)c * x.nseg;
    const int tid = threadIdx.x;
    const uint32_t per = (tiles + gridDim.x - 1) / gridDim.x;
    const uint32_t g0 = blockIdx.x * per, g1 = g0 + per < tiles ? g0 + per : tiles;
    for (int i = tid; i < D * kRadix; i += kSegTileThreads) (&cnt[0][0])[i] = 0;
    uint32_t qcur = 0xFFFFFFFFu;
    auto flush = [&](uint32_t q) {
        uint32_t* h = x.hist + (uint64_t)q * 8 * kRadix;
        for (int i = tid; i < D * kRadix; i += kSegTileThreads) {
            const uint32_t v = (&cnt[0][0])[i];
            if (v) atomicAdd(&h[i], v);
            (&cnt[0][0])[i] = 0;
        }
    };
    for (uint32_t g = g0; g < g1; ++g) {
        __syncthreads();
        const uint32_t q = x.tile_seg[g];
        if (q != qcur) {
            if (qcur != 0xFFFFFFFFu) flush(qcur);
            qcur = q;
            __syncthreads();
        }
        const fs_segment d = x.segs[list[q]];
        const uint64_t t = g - x.tile_prefix[q];
        const uint64_t b0 = t * kSegTile;
        const uint32_t count = (uint32_t)((d.n - b0) < kSegTile ? (d.n - b0) : kSegTile);
        const K* kin = static_cast<const K*>(d.keys_in) + b0;
        for (uint32_t i = tid; i < count; i += kSegTileThreads) {
            const K k = __builtin_nontemporal_load(&kin[i]);
#pragma unroll
            for (int j = 0; j < D; ++j) atomicAdd(&cnt[j][digit_of<K>(k, 8 * j)], 1u);
        }
    }
    __syncthreads();
    if (qcur != 0xFFFFFFFFu) flush(qcur);
    (void)s_q;
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
template <typename K, typename V>
__global__ __launch_bounds__(kSegTileThreads) void k_seg_scatter(SegCtx x, int c, int j) {
    constexpr int W = kSegTileThreads / kWave;
    constexpr int T = (int)kSegTile;
    constexpr int ITEMS = kSegTileItems;
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
    const uint32_t* list = x.large_list + (uint64_t)c * x.nseg;
    const uint32_t epoch = (uint32_t)(1 + 8 * c + j) << (kSegCountBits + 2);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int shift = 8 * j;
    for (int i = tid; i < W * kRadix; i += kSegTileThreads) (&s_peers[0][0])[i] = 0;
    uint32_t* ticket = &x.ctr[ctr_ticket(c, j)];

    for (;;) {
        __syncthreads();
        if (tid == 0) s_ticket = add_agent(ticket, 1u);
        __syncthreads();
        const uint32_t g = s_ticket;
        if (g >= tiles) break;
        const uint32_t q = x.tile_seg[g];
        const uint32_t pl = x.plan[(uint64_t)q * 9 + j];
        if (!(pl & 1u)) continue;  // trivial digit of this segment
        const fs_segment d = x.segs[list[q]];
        const uint32_t t = g - x.tile_prefix[q];
        const uint32_t src = (pl >> 4) & 15u, dstsel = (pl >> 8) & 15u;
        const uint64_t eo = x.elem_prefix[q];
        const K* src_k = src == kBufIn ? static_cast<const K*>(d.keys_in)
                       : src == kBufOut ? static_cast<const K*>(d.keys_out)
                                        : reinterpret_cast<const K*>(x.tmp_k) + eo;
        K* dst_k = dstsel == kBufOut ? static_cast<K*>(d.keys_out) : reinterpret_cast<K*>(x.tmp_k) + eo;
        const VS* src_v = nullptr;
        VS* dst_v = nullptr;
        if constexpr (kHasVals) {
            src_v = src == kBufIn ? static_cast<const VS*>(d.vals_in)
                  : src == kBufOut ? static_cast<const VS*>(d.vals_out)
                                   : reinterpret_cast<const VS*>(x.tmp_v) + eo;
            dst_v = dstsel == kBufOut ? static_cast<VS*>(d.vals_out) : reinterpret_cast<VS*>(x.tmp_v) + eo;
        }
        const uint64_t tb = (uint64_t)t * T;
        const uint32_t count = (uint32_t)((d.n - tb) < (uint64_t)T ? (d.n - tb) : (uint64_t)T);
        const uint32_t wbase = (uint32_t)wave * kWave * ITEMS;
        K key[ITEMS];
        VS val[ITEMS];
#pragma unroll
        for (int k = 0; k < ITEMS; ++k) {
            const uint32_t idx = wbase + k * kWave + lane;
            if (idx < count) {
                key[k] = src_k[tb + idx];
                if constexpr (kHasVals) val[k] = src_v[tb + idx];
            }
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
        const int b = tid;
        uint32_t h = 0;
        for (int w = 0; w < W; ++w) h += s_wcnt[w][b];
        uint32_t* st = x.state + (uint64_t)g * kRadix;
        st_agent(&st[b], epoch | (t == 0 ? kSegPrefix : kSegAgg) | h);
        uint64_t tot;
        const uint32_t start = (uint32_t)scan256_exclusive<uint64_t>(h, s_wsum, &tot);
        {
            uint32_t r = start;
            for (int w = 0; w < W; ++w) {
                const uint32_t cc = s_wcnt[w][b];
                s_wcnt[w][b] = r;
                r += cc;
            }
        }
        uint32_t excl = 0;
        if (t > 0) {
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
        const uint64_t gb = (uint64_t)x.hist[(uint64_t)q * 8 * kRadix + j * kRadix + b] + excl;
        s_delta[b] = gb - start;
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
            const uint32_t qq = k * kSegTileThreads + tid;
            if (qq < count) {
                const K kk = s_keys[qq];
                const uint64_t o = s_delta[digit_of<K>(kk, shift)] + qq;
                if (o < d.n) {
                    dst_k[o] = kk;
                    if constexpr (kHasVals) dst_v[o] = s_vals[qq];
                } else {
                    atomicOr(x.err, 8u);
                }
            }
        }
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
        const uint64_t tb = (uint64_t)(g - x.tile_prefix[q]) * kSegTile;
        const uint64_t te = tb + kSegTile < d.n ? tb + kSegTile : d.n;
        for (uint64_t i = tb + threadIdx.x; i < te; i += 256) {
            static_cast<K*>(d.keys_out)[i] = static_cast<const K*>(d.keys_in)[i];
            if constexpr (kHasVals) static_cast<V*>(d.vals_out)[i] = static_cast<const V*>(d.vals_in)[i];
        }
    }
}

__global__ void k_seg_zero_hist(SegCtx x, int c) {
    const uint64_t words = (uint64_t)x.ctr[ctr_large(c)] * 8 * kRadix;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < words; i += (uint64_t)gridDim.x * blockDim.x)
        x.hist[i] = 0;
}

// ---------------------------------------------------------------------------
template <typename K, typename V>
static hipError_t run_class(const SegCtx& x, int c, int persistent, hipStream_t s) {
    k_seg_zero_hist<<<1024, 256, 0, s>>>(x, c);
    k_seg_layout<<<1, 1024, 0, s>>>(x, c);
    k_seg_tilemap<<<256, 256, 0, s>>>(x, c);
    k_seg_hist<K><<<persistent, kSegTileThreads, 0, s>>>(x, c);
    k_seg_scan<K><<<persistent, 256, 0, s>>>(x, c);
    for (int j = 0; j < (int)sizeof(K); ++j) k_seg_scatter<K, V><<<persistent, kSegTileThreads, 0, s>>>(x, c, j);
    k_seg_copy<K, V><<<persistent, 256, 0, s>>>(x, c);
    return hipGetLastError();
}

uint32_t seg_max_tiles(uint64_t total_keys, uint32_t nseg) {
    return (uint32_t)(total_keys / kSegTile + nseg + 1);
}

hipError_t launch_segmented(const SegCtx& x, hipStream_t s) {
    const int cus = device_cu_count();
    k_seg_classify<<<(x.nseg + 255) / 256 < 1024 ? (x.nseg + 255) / 256 : 1024, 256, 0, s>>>(x);
    k_seg_small<<<cus * 2, kSmallThreads, 0, s>>>(x);
    const int P = cus * 2;
    hipError_t e;
    if ((e = run_class<uint16_t, NoVal>(x, 0, P, s)) != hipSuccess) return e;
    if ((e = run_class<uint16_t, uint32_t>(x, 1, P, s)) != hipSuccess) return e;
    if ((e = run_class<uint16_t, uint64_t>(x, 2, P, s)) != hipSuccess) return e;
    if ((e = run_class<uint32_t, NoVal>(x, 3, P, s)) != hipSuccess) return e;
    if ((e = run_class<uint32_t, uint32_t>(x, 4, P, s)) != hipSuccess) return e;
    if ((e = run_class<uint32_t, uint64_t>(x, 5, P, s)) != hipSuccess) return e;
    if ((e = run_class<uint64_t, NoVal>(x, 6, P, s)) != hipSuccess) return e;
    if ((e = run_class<uint64_t, uint32_t>(x, 7, P, s)) != hipSuccess) return e;
    return run_class<uint64_t, uint64_t>(x, 8, P, s);
}

}  // namespace fs
