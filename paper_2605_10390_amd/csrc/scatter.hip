// One stable LSD scatter pass over an 8-bit digit, single sweep with
// decoupled look-back.
//
// The paper's stable scatter phase (Section II) moves every key (and its
// payload) to  start[digit] + (number of earlier keys with that digit).  The
// start comes from the exclusive scan of the digit's histogram (the paper's
// GetIndex, Algorithm 3); the "earlier keys" part is split into
// (a) keys of earlier tiles, found by decoupled look-back over per-tile bin
// counts published in global memory, and (b) keys earlier in this tile,
// found per wave: every lane ORs its lane bit into an LDS word kept per
// digit, so reading the word back gives each lane the full set of lanes
// that share its digit (in any order of the atomic ORs), and the lowest of
// them advances the wave's running count for the digit.  The tile is then
// staged in LDS in digit order and written out as contiguous per-digit runs.
//
// Workgroups are persistent and take tiles from an ordered ticket counter,
// so a tile only ever waits for tiles that are already running; every wait
// is bounded (kSpinLimit) and raises the workspace error word if exceeded.
#include "fs_device.hpp"
#include "fs_internal.hpp"

namespace fs {

// predecessor tiles whose states one look-back round reads at once
constexpr int kLookbackWindow = 16;

template <typename K, typename V, int THREADS, int ITEMS>
__global__ __launch_bounds__(THREADS) void k_scatter(ScatterArgs a) {
    constexpr int W = THREADS / kWave;
    constexpr int T = THREADS * ITEMS;
    constexpr bool kHasVals = !__is_same(V, NoVal);
    using VS = typename std::conditional<kHasVals, V, uint32_t>::type;
    static_assert(THREADS >= kRadix, "one thread per digit value in the look-back");

    __shared__ uint64_t s_peers[W][kRadix];  // lanes holding each digit in the current item
    __shared__ uint32_t s_wcnt[W][kRadix];   // per-wave running counts, then tile offsets
    __shared__ uint64_t s_delta[kRadix];     // global destination of tile slot q is s_delta[d] + q
    __shared__ uint64_t s_wsum[4];
    __shared__ uint32_t s_ticket;
    __shared__ K s_keys[T];
    __shared__ VS s_vals[kHasVals ? T : 1];

    if (!a.plan[4 * a.pass]) return;  // trivial digit: pass skipped
    const uint32_t src_sel = a.plan[4 * a.pass + 1], dst_sel = a.plan[4 * a.pass + 2];
    const K* src_k = static_cast<const K*>(src_sel == kBufIn ? a.in_k : src_sel == kBufOut ? a.out_k : a.tmp_k);
    K* dst_k = static_cast<K*>(dst_sel == kBufOut ? a.out_k : a.tmp_k);
    const VS* src_v = nullptr;
    VS* dst_v = nullptr;
    if constexpr (kHasVals) {
        src_v = static_cast<const VS*>(src_sel == kBufIn ? a.in_v : src_sel == kBufOut ? a.out_v : a.tmp_v);
        dst_v = static_cast<VS*>(dst_sel == kBufOut ? a.out_v : a.tmp_v);
    }

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const uint64_t lane_bit = 1ull << lane;
    const uint64_t portion_end = a.portion_begin + a.portion_len;
    for (int i = tid; i < W * kRadix; i += THREADS) (&s_peers[0][0])[i] = 0;

    for (;;) {
        if (tid == 0) s_ticket = add_agent(a.ticket, 1u);
        __syncthreads();
        const uint32_t t = s_ticket;
        if (t >= a.tiles) break;
        const uint64_t tile_begin = a.portion_begin + (uint64_t)t * T;
        const uint32_t count = (uint32_t)((portion_end - tile_begin) < (uint64_t)T ? (portion_end - tile_begin) : T);

        // ---- load: wave w owns slots [w*64*ITEMS, (w+1)*64*ITEMS), item k of
        //      lane l is slot w*64*ITEMS + k*64 + l (input order = (w, k, l))
        K key[ITEMS];
        VS val[ITEMS];
        const uint32_t wbase = (uint32_t)wave * kWave * ITEMS;
#pragma unroll
        for (int k = 0; k < ITEMS; ++k) {
            const uint32_t idx = wbase + k * kWave + lane;
            if (idx < count) {
                key[k] = __builtin_nontemporal_load(&src_k[tile_begin + idx]);
                if constexpr (kHasVals) val[k] = __builtin_nontemporal_load(&src_v[tile_begin + idx]);
            }
        }
#pragma unroll
        for (int i = 0; i < kRadix / kWave; ++i) s_wcnt[wave][lane + kWave * i] = 0;
        __builtin_amdgcn_wave_barrier();

        // ---- rank inside the wave: lanes below with the same digit, plus this
        //      wave's count of the digit in earlier items
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

        // ---- per digit (thread b < 256): tile count, publish, scan, look back
        const int b = tid;
        uint32_t h = 0;
        if (b < kRadix) {
#pragma unroll
            for (int w = 0; w < W; ++w) h += s_wcnt[w][b];
            st_agent(&a.state[(uint64_t)t * kRadix + b], (t == 0 ? kFlagPrefix : kFlagAggregate) | h);
        }
        uint64_t tile_total;
        const uint32_t start = (uint32_t)scan256_exclusive<uint64_t>(b < kRadix ? h : 0, s_wsum, &tile_total);
        if (b < kRadix) {
            // wave offsets become tile offsets: slot of a key = s_wcnt[w][d] + rank
            uint32_t run = start;
#pragma unroll
            for (int w = 0; w < W; ++w) {
                const uint32_t c = s_wcnt[w][b];
                s_wcnt[w][b] = run;
                run += c;
            }
            uint32_t excl = 0;
            if (t > 0) {
                int64_t j = (int64_t)t - 1;  // nearest tile not yet folded in
                uint32_t spins = 0;
                bool done = false;
                while (!done) {
                    uint32_t sw[kLookbackWindow];
#pragma unroll
                    for (int i = 0; i < kLookbackWindow; ++i)
                        sw[i] = (j - i >= 0) ? ld_agent(&a.state[(uint64_t)(j - i) * kRadix + b]) : kFlagPrefix;
#pragma unroll
                    for (int i = 0; i < kLookbackWindow; ++i) {
                        if (done) break;
                        uint32_t w = sw[i];
                        while ((w & ~kCountMask) == 0) {  // predecessor not published yet
                            if (++spins > kSpinLimit) {
                                atomicOr(a.err, 1u);
                                w = kFlagPrefix;
                                break;
                            }
                            __builtin_amdgcn_s_sleep(1);
                            w = ld_agent(&a.state[(uint64_t)(j - i) * kRadix + b]);
                        }
                        excl += w & kCountMask;
                        done = (w & kFlagPrefix) != 0;
                    }
                    j -= kLookbackWindow;
                    if (!done && j < 0) {  // tile 0 always publishes a prefix
                        atomicOr(a.err, 2u);
                        done = true;
                    }
                }
                st_agent(&a.state[(uint64_t)t * kRadix + b], kFlagPrefix | (excl + h));
            }
            const uint64_t gbase = a.base_cur[b] + excl;
            s_delta[b] = gbase - start;
            if (t == a.tiles - 1) a.base_next[b] = gbase + h;
        }
        __syncthreads();

        // ---- stage the tile in LDS in digit order
#pragma unroll
        for (int k = 0; k < ITEMS; ++k) {
            if (wbase + k * kWave + lane < count) {
                const uint32_t pos = s_wcnt[wave][digit_of<K>(key[k], a.shift)] + rank[k];
                if (pos < (uint32_t)T) {
                    s_keys[pos] = key[k];
                    if constexpr (kHasVals) s_vals[pos] = val[k];
                } else {
                    atomicOr(a.err, 4u);
                }
            }
        }
        __syncthreads();

        // ---- write contiguous per-digit runs
#pragma unroll
        for (int k = 0; k < ITEMS; ++k) {
            const uint32_t q = k * THREADS + tid;
            if (q < count) {
                const K kk = s_keys[q];
                const uint64_t dst = s_delta[digit_of<K>(kk, a.shift)] + q;
                if (dst < a.n) {
                    __builtin_nontemporal_store(kk, &dst_k[dst]);
                    if constexpr (kHasVals) __builtin_nontemporal_store(s_vals[q], &dst_v[dst]);
                } else {
                    atomicOr(a.err, 8u);
                }
            }
        }
        __syncthreads();
    }
}

#ifndef FS_SCATTER_THREADS
#define FS_SCATTER_THREADS 256
#endif
#ifndef FS_SCATTER_ITEMS
#define FS_SCATTER_ITEMS 16
#endif

ScatterShape scatter_shape(int key_bytes, int val_bytes) {
    (void)key_bytes;
    (void)val_bytes;
    return ScatterShape{FS_SCATTER_THREADS, FS_SCATTER_ITEMS};
}

template <typename K, typename V>
static hipError_t launch_kv(const ScatterArgs& a, hipStream_t s) {
    constexpr int THREADS = FS_SCATTER_THREADS, ITEMS = FS_SCATTER_ITEMS;
    static int grid = 0;
    if (grid == 0) {
        int per_cu = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_scatter<K, V, THREADS, ITEMS>, THREADS, 0) !=
                hipSuccess ||
            per_cu < 1)
            per_cu = 1;
        grid = per_cu * device_cu_count();
    }
    unsigned g = (unsigned)(a.tiles < (uint32_t)grid ? a.tiles : (uint32_t)grid);
    if (g == 0) g = 1;
    k_scatter<K, V, THREADS, ITEMS><<<g, THREADS, 0, s>>>(a);
    return hipGetLastError();
}

hipError_t launch_scatter(const ScatterArgs& a, int key_bytes, int val_bytes, hipStream_t s) {
    switch (key_bytes * 16 + val_bytes) {
    case 2 * 16 + 0: return launch_kv<uint16_t, NoVal>(a, s);
    case 2 * 16 + 4: return launch_kv<uint16_t, uint32_t>(a, s);
    case 2 * 16 + 8: return launch_kv<uint16_t, uint64_t>(a, s);
    case 4 * 16 + 0: return launch_kv<uint32_t, NoVal>(a, s);
    case 4 * 16 + 4: return launch_kv<uint32_t, uint32_t>(a, s);
    case 4 * 16 + 8: return launch_kv<uint32_t, uint64_t>(a, s);
    case 8 * 16 + 0: return launch_kv<uint64_t, NoVal>(a, s);
    case 8 * 16 + 4: return launch_kv<uint64_t, uint32_t>(a, s);
    case 8 * 16 + 8: return launch_kv<uint64_t, uint64_t>(a, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace fs
