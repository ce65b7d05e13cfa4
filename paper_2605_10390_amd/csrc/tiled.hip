// Stable LSD sort by reduce-then-scan over fixed tiles, with no waiting
// between workgroups.
//
// The paper builds a histogram of narrow counters once per batch (Section
// III-A/B, Algorithm 1; counter width tapered to the batch, Section
// III-D.1) and reads positions back as prefix sums (GetIndex, Algorithm 3).
// Here a batch is a tile of T keys.  Each pass of one 8-bit digit runs three
// steps:
//
//   1. tile histograms: for every tile, the 256 counts of the pass digit as
//      packed 16-bit counters (T < 2^16, so a tile's counters cannot wrap),
//      turned at once into prefixes inside blocks of tiles; the first pass
//      also accumulates every digit's global counts for the pass plan;
//   2. offsets: the remaining levels of the exclusive prefix of every digit
//      over the tiles, added to the digit's start in the pass output (the
//      plan's exclusive scan);
//   3. scatter: each tile is ranked per wave, staged in LDS in digit order
//      and written as contiguous per-digit runs starting at its offsets.
//
// Write locality: the tiles are split into 8 contiguous groups, one per
// XCD (workgroup g of a launch runs on XCD g mod 8), and the workgroups of a
// group walk their group's tiles in order.  So the tiles in flight on one
// XCD at any time are consecutive, their runs of every digit are adjacent in
// the output, and the cache lines that two runs share meet in that XCD's L2
// and leave it whole.  The split only steers performance: every offset is
// precomputed, so results do not depend on where a workgroup runs.
#include "fs_device.hpp"
#include "fs_internal.hpp"
#include "fs_plan.hpp"

#include <type_traits>

namespace fs {

constexpr int kTileHistThreads = 512;

template <typename K>
__device__ __forceinline__ const K* pass_source(const TiledArgs& a, uint32_t sel) {
    return static_cast<const K*>(sel == kBufIn ? a.in_k : sel == kBufOut ? a.out_k : a.tmp_k);
}

// ---------------------------------------------------------------------------
// Step 1: tile histograms and the first offset level.
//
// A block is 65536 / T consecutive tiles; every histogram workgroup owns a
// contiguous run of whole blocks and walks it in order, a few tiles per
// step (all of a step's loads are issued before its counting).  The counts of a tile are kept in LDS as packed 16-bit counters
// (bins 2w and 2w+1 in word w; a tile holds at most T < 2^16 keys, so the
// halves cannot carry), one copy per wave parity and tile of the step, and
// double-buffered between steps so that one barrier per step suffices.
// The workgroup then writes, per tile t and digit value d,
//   th[t][d]   = counts of d in the tiles of t's block before t  (16 bits,
//                packed in pairs like the counters: at most 65536 - T)
//   bsum[b][d] = total count of d in block b.
// With FIRST the workgroup also counts every other digit of its keys, and
// part[g][j][b] receives its totals of digit j == b for the pass plan.
// ---------------------------------------------------------------------------
constexpr int kHistCopies = 2;
// 16-byte vectors per thread and step (plus one for misalignment): two for
// one-byte keys, whose 16 keys a vector each would otherwise hold too many
// registers
template <typename K>
constexpr int hist_vecs() { return sizeof(K) == 1 ? 2 : 4; }

template <typename K, bool FIRST, int TILE, bool ORD>
__global__ __launch_bounds__(kTileHistThreads) void k_tile_hist(TiledArgs a, int pass) {
    constexpr int D = sizeof(K);
    constexpr int VK = 16 / sizeof(K);
    constexpr int DX = FIRST ? D : 1;  // digits counted per workgroup (index 0 unused)
    constexpr int SETW = kRadix / 2;   // words of one packed tile histogram
    constexpr int kHistVecs = hist_vecs<K>();
    constexpr int TPS = kHistVecs * kTileHistThreads * VK / TILE;  // tiles per step
    static_assert(TPS >= 1 && TPS * TILE == kHistVecs * kTileHistThreads * VK, "whole tiles per step");
    __shared__ uint32_t s_t[2][TPS][kHistCopies][SETW];
    __shared__ uint32_t s_all[DX][kRadix];

    const K* src;
    int shift = 0;  // the first read counts digit 0's tiles
    if constexpr (FIRST) {
        src = static_cast<const K*>(a.in_k);
    } else {
        if (!a.plan[4 * pass]) return;
        // slot 0 is counted by the first read unless it sorts another digit
        if (pass == 0 && !a.plan[kPlanRecount0]) return;
        src = pass_source<K>(a, a.plan[4 * pass + 1]);
        // one-byte keys have a single digit (shift 0)
        shift = sizeof(K) == 1 ? 0 : 8 * (int)a.plan[4 * pass + 3];
        if (sizeof(K) == 1 && a.narrow) src = reinterpret_cast<const K*>(a.narrow);  // 16-bit pairs' second pass
    }
    const int tid = threadIdx.x, wave = tid >> 6, copy = wave % kHistCopies;
    for (int i = tid; i < 2 * TPS * kHistCopies * SETW; i += kTileHistThreads) (&s_t[0][0][0][0])[i] = 0;
    for (int i = tid; i < DX * kRadix; i += kTileHistThreads) (&s_all[0][0])[i] = 0;

    const uint64_t blocks = (a.tiles + a.block_tiles - 1) / a.block_tiles;
    const uint64_t blo = blocks * blockIdx.x / gridDim.x, bhi = blocks * (blockIdx.x + 1) / gridDim.x;
    const uint64_t tlo = blo * a.block_tiles;
    const uint64_t thi = bhi * a.block_tiles < a.tiles ? bhi * a.block_tiles : a.tiles;
    const uint32_t head = (uint32_t)((reinterpret_cast<uintptr_t>(src) & 15) / sizeof(K));

    // thread w < 128 owns bins 2w and 2w+1: running counts inside the
    // current block and workgroup totals
    uint32_t run_lo = 0, run_hi = 0, tot_lo = 0, tot_hi = 0;
    int par = 0;
    __syncthreads();
    for (uint64_t t0 = tlo; t0 < thi; t0 += TPS, par ^= 1) {
        const uint64_t lo = t0 * TILE;
        const uint64_t hi_t = t0 + TPS < thi ? t0 + TPS : thi;
        const uint64_t hi = hi_t * TILE < a.n ? hi_t * TILE : a.n;
        const uint32_t cnt = (uint32_t)(hi - lo);
        // the step's keys [lo, hi) lie in the aligned vectors starting at key
        // index lo - sh
        const uint32_t sh = each_iteration((uint32_t)((lo + head) % VK));
        const uint32_t nv = (sh + cnt + VK - 1) / VK;
        const u32x4* gv = reinterpret_cast<const u32x4*>(src + (lo - sh));
        // all of the step's loads first, then the counting
        // unconditional loads at a clamped index (lanes past the step's last
        // vector reload it and never count it), so no guard branch makes
        // the compiler wait for each load before issuing the next
        u32x4 q[kHistVecs + 1];
#pragma unroll
        for (int r = 0; r <= kHistVecs; ++r) {
            const uint32_t v = tid + r * kTileHistThreads;
            q[r] = __builtin_nontemporal_load(&gv[v < nv ? v : nv - 1]);
        }
        if constexpr (ORD) {  // count the mapped keys (order_map)
#pragma unroll
            for (int r = 0; r <= kHistVecs; ++r) q[r] = order_map_vec<K>(q[r], a.ord_pos, a.ord_neg);
        }
        // skewed digits: is the digit of the wave's first key shared by at
        // least kSkewLanes lanes in the step's first vector?  (wave-uniform;
        // spread keys then count exactly as without the check.)  Bit j of
        // skew_all answers it for digit j of the first pass's totals.
        bool skewed = false;
        uint32_t skew_all = 0;
        uint32_t hot = 0;  // the step's leading digit (when skewed)
        {
            const uint32_t v = tid;
            const bool in0 = v < nv && (int32_t)(v * VK) - (int32_t)sh >= 0;
            K k0[VK];
            __builtin_memcpy(k0, &q[0], 16);
            const uint32_t d0 = digit_of<K>(k0[0], shift);
            const uint32_t lead = __builtin_amdgcn_readfirstlane(in0 ? d0 : 0xFFFFFFFFu);
            skewed = popc64(ballot(in0 && d0 == lead)) >= kSkewLanes;
            hot = lead;
            if constexpr (FIRST) {
#pragma unroll
                for (int j = 1; j < D; ++j) {
                    const uint32_t dj = digit_of<K>(k0[0], 8 * j);
                    const uint32_t lj = __builtin_amdgcn_readfirstlane(in0 ? dj : 0xFFFFFFFFu);
                    if (popc64(ballot(in0 && dj == lj)) >= kSkewLanes) skew_all |= 1u << j;
                }
            }
        }
        // the first pass's totals of digit j for one element (leader
        // aggregation when that digit is skewed in this step)
        auto count_all = [&](const K key, bool in) {
            if constexpr (FIRST) {
#pragma unroll
                for (int j = 1; j < D; ++j) {
                    const uint32_t dj = digit_of<K>(key, 8 * j);
                    if ((skew_all >> j) & 1u) {
                        uint32_t shared;
                        const uint32_t c = leader_count(dj, in, &shared);
                        if (c) atomicAdd(&s_all[j][dj], c);
                    } else if (in) {
                        atomicAdd(&s_all[j][dj], 1u);
                    }
                }
            }
        };
#pragma unroll
        for (int r = 0; r <= kHistVecs; ++r) {
            const uint32_t v = tid + r * kTileHistThreads;
            if (r == kHistVecs && __builtin_amdgcn_readfirstlane(v) >= nv) break;  // wave-uniform
            if (v < nv) {
                K k[VK];
                __builtin_memcpy(k, &q[r], 16);
                // step index of element e is first + e (negative in a head vector)
                const int32_t first = (int32_t)(v * VK) - (int32_t)sh;
                const bool whole = first >= 0 && first + VK <= (int32_t)cnt &&
                                   (uint32_t)first / TILE == (uint32_t)(first + VK - 1) / TILE;
                const uint64_t active = ballot(true);
                const uint64_t kw =
                    ((uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)k[0] >> 32)) << 32) |
                    __builtin_amdgcn_readfirstlane((uint32_t)(uint64_t)k[0]);
                if (!skewed && ballot(whole) == active && ballot((uint64_t)k[0] == kw) != active) {
                    // spread digits, every lane's vector inside the step and
                    // inside one tile: an add of one per key
                    uint32_t* tc = &s_t[par][(uint32_t)first / TILE][copy][0];
#pragma unroll
                    for (int e = 0; e < VK; ++e) {
                        const uint32_t d = digit_of<K>(k[e], shift);
                        atomicAdd(&tc[d >> 1], 1u << ((d & 1u) << 4));
                    }
#pragma unroll
                    for (int e = 0; e < VK; ++e) count_all(k[e], true);
                    __builtin_amdgcn_sched_barrier(0);
                    continue;
                }
                bool same = whole;
#pragma unroll
                for (int e = 1; e < VK; ++e) same &= k[e] == k[0];
                // one add for a whole wave holding one key value inside one tile
                const uint32_t set0 = whole ? (uint32_t)first / TILE : 0xFFFFFFFFu;
                const uint32_t setw = __builtin_amdgcn_readfirstlane(set0);
                if (ballot(same && (uint64_t)k[0] == kw && set0 == setw) == active) {
                    if (lanes_below(active) == 0) {
                        const uint32_t c = (uint32_t)VK * popc64(active);
                        const uint32_t d = digit_of<uint64_t>(kw, shift);
                        atomicAdd(&s_t[par][setw][copy][d >> 1], c << ((d & 1) * 16));
                        if constexpr (FIRST) {
#pragma unroll
                            for (int j = 1; j < D; ++j) atomicAdd(&s_all[j][digit_of<uint64_t>(kw, 8 * j)], c);
                        }
                    }
                } else if (VK >= 8 && skewed && active == ~0ull && ballot(whole && set0 == setw) == active) {
                    // skewed digits of keys of up to 16 bits, the whole wave
                    // inside one tile: each lane counts its keys holding the
                    // step's leading digit and the wave sums those counts
                    // (across all 64 lanes) into one add; other keys add one
                    // each.  (Wider keys, 4 or 2 per vector, do not repay
                    // the wave sum and take the leader path.)
                    uint32_t* tc = &s_t[par][setw][copy][0];
                    uint32_t nh = 0;
#pragma unroll
                    for (int e = 0; e < VK; ++e) {
                        const uint32_t d = digit_of<K>(k[e], shift);
                        if (d == hot) ++nh;
                        else atomicAdd(&tc[d >> 1], 1u << ((d & 1u) << 4));
                    }
#pragma unroll
                    for (int e = 0; e < VK; ++e) count_all(k[e], true);
#pragma unroll
                    for (int o = 32; o >= 1; o >>= 1) nh += __shfl_xor(nh, o, 64);
                    if (lanes_below(active) == 0 && nh) atomicAdd(&tc[hot >> 1], nh << ((hot & 1u) << 4));
                } else if (skewed) {
                    // lanes sharing the leader's (tile, digit) add once
#pragma unroll
                    for (int e = 0; e < VK; ++e) {
                        const int32_t idx = first + e;
                        const bool in = idx >= 0 && idx < (int32_t)cnt;
                        const uint32_t d = digit_of<K>(k[e], shift);
                        const uint32_t set = in ? (uint32_t)idx / TILE : 0u;
                        uint32_t shared;
                        const uint32_t c = leader_count((set << 8) | d, in, &shared);
                        if (c) atomicAdd(&s_t[par][set][copy][d >> 1], c << ((d & 1) * 16));
                        count_all(k[e], in);
                    }
                } else {
#pragma unroll
                    for (int e = 0; e < VK; ++e) {
                        const int32_t idx = first + e;
                        const bool in = idx >= 0 && idx < (int32_t)cnt;
                        if (in) {
                            const uint32_t d = digit_of<K>(k[e], shift);
                            atomicAdd(&s_t[par][(uint32_t)idx / TILE][copy][d >> 1], 1u << ((d & 1) * 16));
                        }
                        if constexpr (FIRST) {
                            if (skew_all) count_all(k[e], in);
                            else if (in) {
#pragma unroll
                                for (int j = 1; j < D; ++j) atomicAdd(&s_all[j][digit_of<K>(k[e], 8 * j)], 1u);
                            }
                        }
                    }
                }
            }
            __builtin_amdgcn_sched_barrier(0);  // count one vector at a time (register pressure)
        }
        __syncthreads();
        // each counter word has one reader, which also clears it for the
        // step after next (the next step counts into the other parity)
        if (tid < SETW) {
            const uint32_t w = tid;
            for (uint64_t t = t0; t < hi_t; ++t) {
                const uint32_t set = (uint32_t)(t - t0);
                uint32_t c = 0;
#pragma unroll
                for (int i = 0; i < kHistCopies; ++i) {
                    c += s_t[par][set][i][w];  // halves cannot carry: each is at most TILE < 2^16
                    s_t[par][set][i][w] = 0;
                }
                a.th[t * SETW + w] = run_lo | (run_hi << 16);
                run_lo += c & 0xFFFFu;
                run_hi += c >> 16;
                tot_lo += c & 0xFFFFu;
                tot_hi += c >> 16;
                if ((t + 1) % a.block_tiles == 0 || t + 1 == a.tiles) {
                    uint32_t* bs = a.bsum + (t / a.block_tiles) * kRadix;
                    bs[2 * w] = run_lo;
                    bs[2 * w + 1] = run_hi;
                    run_lo = run_hi = 0;
                }
            }
        }
    }
    if constexpr (FIRST) {
        __syncthreads();
        uint32_t* dst = a.part + (uint64_t)blockIdx.x * D * kRadix;
        if (tid < SETW) {
            dst[2 * tid] = tot_lo;
            dst[2 * tid + 1] = tot_hi;
        }
        for (int i = tid; i < (D - 1) * kRadix; i += kTileHistThreads) dst[kRadix + i] = (&s_all[1][0])[i];
    }
}

// ---------------------------------------------------------------------------
// First histogram of a 16-bit pair sort: the compressed 2^16-bin histogram
// of the whole key (Section III-B, Algorithm 1; counters packed two per LDS
// word with exact wrap repair, hist16_add) and, in the same read, the tile
// counts of digit 0 turned into block prefixes as in k_tile_hist.  The
// 2^16-bin histogram gives both digit histograms for the plan (its
// marginals) and, through its prefix, the sorted keys themselves
// (Algorithm 5 with no trailing bits), so the last scatter pass only moves
// the payloads.  One workgroup of kHist16Threads per CU (the counters take
// 128 KiB of LDS).
// ---------------------------------------------------------------------------
template <int TILE, bool ORD>
__global__ __launch_bounds__(kHist16Threads) void k_tile_hist16(TiledArgs a, uint32_t* __restrict__ part16,
                                                                 uint32_t* wrap_lo, uint32_t* wrap_word) {
    using K = uint16_t;
    constexpr int THREADS = kHist16Threads;
    constexpr int VK = 8;
    constexpr int NW = THREADS / kWave;
    constexpr int SETW = kRadix / 2;
    constexpr int HV = 2;  // vectors per thread and step (plus one for misalignment)
    constexpr int TPS = HV * THREADS * VK / TILE;  // tiles per step
    static_assert(TPS >= 1 && TPS * TILE == HV * THREADS * VK, "whole tiles per step");
    __shared__ uint32_t cnt[kHist16Words];
    __shared__ uint32_t s_t[2][TPS][kHistCopies][SETW];

    const K* src = static_cast<const K*>(a.in_k);
    const int tid = threadIdx.x, wave = tid >> 6, copy = wave % kHistCopies;
    for (int i = tid; i < kHist16Words; i += THREADS) cnt[i] = 0;
    for (int i = tid; i < 2 * TPS * kHistCopies * SETW; i += THREADS) (&s_t[0][0][0][0])[i] = 0;

    const uint64_t blocks = (a.tiles + a.block_tiles - 1) / a.block_tiles;
    const uint64_t blo = blocks * blockIdx.x / gridDim.x, bhi = blocks * (blockIdx.x + 1) / gridDim.x;
    const uint64_t tlo = blo * a.block_tiles;
    const uint64_t thi = bhi * a.block_tiles < a.tiles ? bhi * a.block_tiles : a.tiles;
    const uint32_t head = (uint32_t)((reinterpret_cast<uintptr_t>(src) & 15) / sizeof(K));
    uint32_t run_lo = 0, run_hi = 0;  // thread w < 128: bins 2w, 2w+1 of digit 0 inside the block
    int par = 0;
    (void)NW;
    __syncthreads();
    // a step's vectors, loaded one step ahead
    u32x4 qn[HV + 1];
    auto load_step = [&](uint64_t t) {
        const uint64_t l = t * TILE;
        const uint64_t ht = t + TPS < thi ? t + TPS : thi;
        const uint64_t h = ht * TILE < a.n ? ht * TILE : a.n;
        const uint32_t c = (uint32_t)(h - l);
        const uint32_t s0 = (uint32_t)((l + head) % VK);
        const uint32_t m = (s0 + c + VK - 1) / VK;
        const u32x4* g = reinterpret_cast<const u32x4*>(src + (l - s0));
#pragma unroll
        for (int r = 0; r <= HV; ++r) {
            const uint32_t v = tid + r * THREADS;
            if (v < m) qn[r] = __builtin_nontemporal_load(&g[v]);
        }
    };
    if (tlo < thi) load_step(tlo);
    for (uint64_t t0 = tlo; t0 < thi; t0 += TPS, par ^= 1) {
        const uint64_t lo = t0 * TILE;
        const uint64_t hi_t = t0 + TPS < thi ? t0 + TPS : thi;
        const uint64_t hi = hi_t * TILE < a.n ? hi_t * TILE : a.n;
        const uint32_t cntk = (uint32_t)(hi - lo);
        const uint32_t sh = each_iteration((uint32_t)((lo + head) % VK));
        const uint32_t nv = (sh + cntk + VK - 1) / VK;
        u32x4 q[HV + 1];
#pragma unroll
        for (int r = 0; r <= HV; ++r) q[r] = qn[r];
        // the next step's vectors are requested now, in flight while this
        // step is counted
        if (t0 + TPS < thi) load_step(t0 + TPS);
        if constexpr (ORD) {  // count the mapped keys (order_map)
#pragma unroll
            for (int r = 0; r <= HV; ++r)
                if (tid + r * THREADS < nv) q[r] = order_map_vec<K>(q[r], a.ord_pos, a.ord_neg);
        }
#pragma unroll
        for (int r = 0; r <= HV; ++r) {
            const uint32_t v = tid + r * THREADS;
            if (r == HV && __builtin_amdgcn_readfirstlane(v) >= nv) break;  // wave-uniform
            if (v < nv) {
                K k[VK];
                __builtin_memcpy(k, &q[r], 16);
                const int32_t first = (int32_t)(v * VK) - (int32_t)sh;
                const bool whole = first >= 0 && first + VK <= (int32_t)cntk &&
                                   (uint32_t)first / TILE == (uint32_t)(first + VK - 1) / TILE;
                const uint64_t active = ballot(true);
                const uint32_t kw = __builtin_amdgcn_readfirstlane((uint32_t)k[0]);
                const uint64_t lead = ballot((uint32_t)k[0] == kw);
                if (popc64(lead) < kSkewLanes && ballot(whole) == active) {
                    // spread keys, every lane's vector inside the step and
                    // inside one tile: an add of one per key, in the
                    // histogram and in the tile's digit-0 counts
                    uint32_t kk[VK];
#pragma unroll
                    for (int e = 0; e < VK; ++e) kk[e] = k[e];
                    hist16_add_ones<VK>(cnt, kk, &s_t[par][(uint32_t)first / TILE][copy][0], wrap_lo, wrap_word);
                } else {
                    bool same = whole;
#pragma unroll
                    for (int e = 1; e < VK; ++e) same &= k[e] == k[0];
                    const uint32_t set0 = whole ? (uint32_t)first / TILE : 0xFFFFFFFFu;
                    const uint32_t setw = __builtin_amdgcn_readfirstlane(set0);
                    if (ballot(same && (uint32_t)k[0] == kw && set0 == setw) == active) {
                        // a whole wave holding one key value inside one tile: one add each
                        if (lanes_below(active) == 0) {
                            const uint32_t c = (uint32_t)VK * popc64(active);
                            hist16_add(cnt, kw, c, wrap_lo, wrap_word);
                            const uint32_t d = kw & 0xFFu;
                            atomicAdd(&s_t[par][setw][copy][d >> 1], c << ((d & 1) * 16));
                        }
                    } else {
                        // all adds issued before any carry check (hist16_add_n);
                        // keys outside the range add 0; lanes sharing the
                        // leader's (tile, key) add once (checked on the first
                        // element, kept if it paid)
                        uint32_t kk[VK], cc[VK], st[VK];
                        bool skewed = false;
#pragma unroll
                        for (int e = 0; e < VK; ++e) {
                            const int32_t idx = first + e;
                            const bool in = idx >= 0 && idx < (int32_t)cntk;
                            kk[e] = k[e];
                            st[e] = in ? (uint32_t)idx / TILE : 0u;
                            cc[e] = in ? 1u : 0u;
                            if (e == 0 || skewed) {
                                uint32_t shared;
                                cc[e] = leader_count((st[e] << 16) | kk[e], in, &shared);
                                if (e == 0) skewed = shared >= kSkewLanes;
                            }
                        }
                        hist16_add_n<VK>(cnt, kk, cc, wrap_lo, wrap_word);
#pragma unroll
                        for (int e = 0; e < VK; ++e) {
                            const uint32_t d = kk[e] & 0xFFu;
                            if (cc[e]) atomicAdd(&s_t[par][st[e]][copy][d >> 1], cc[e] << ((d & 1) * 16));
                        }
                    }
                }
            }
            __builtin_amdgcn_sched_barrier(0);  // count one vector at a time (register pressure)
        }
        __syncthreads();
        if (tid < SETW) {
            const uint32_t w = tid;
            for (uint64_t t = t0; t < hi_t; ++t) {
                const uint32_t set = (uint32_t)(t - t0);
                uint32_t c = 0;
#pragma unroll
                for (int i = 0; i < kHistCopies; ++i) {
                    c += s_t[par][set][i][w];
                    s_t[par][set][i][w] = 0;
                }
                a.th[t * SETW + w] = run_lo | (run_hi << 16);
                run_lo += c & 0xFFFFu;
                run_hi += c >> 16;
                if ((t + 1) % a.block_tiles == 0 || t + 1 == a.tiles) {
                    uint32_t* bs = a.bsum + (t / a.block_tiles) * kRadix;
                    bs[2 * w] = run_lo;
                    bs[2 * w + 1] = run_hi;
                    run_lo = run_hi = 0;
                }
            }
        }
    }
    __syncthreads();
    uint32_t* dst = part16 + (uint64_t)blockIdx.x * kHist16Words;
    for (int i = tid; i < kHist16Words; i += THREADS) dst[i] = cnt[i];
}

hipError_t launch_tile_hist16(const TiledArgs& a, uint32_t groups, uint32_t* part16, uint32_t* wrap_lo,
                              uint32_t* wrap_word, hipStream_t s) {
    if (a.tile == 8192) {
        if (a.ord_pos | a.ord_neg)
            k_tile_hist16<8192, true><<<groups, kHist16Threads, 0, s>>>(a, part16, wrap_lo, wrap_word);
        else
            k_tile_hist16<8192, false><<<groups, kHist16Threads, 0, s>>>(a, part16, wrap_lo, wrap_word);
        return hipGetLastError();
    }
    if (a.tile != 4096) return hipErrorInvalidValue;
    if (a.ord_pos | a.ord_neg)
        k_tile_hist16<4096, true><<<groups, kHist16Threads, 0, s>>>(a, part16, wrap_lo, wrap_word);
    else
        k_tile_hist16<4096, false><<<groups, kHist16Threads, 0, s>>>(a, part16, wrap_lo, wrap_word);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Pass plan from the first pass's workgroup totals: every digit's global
// counts, their exclusive scans and the trivial digits (finish_plan).  One
// block of kPlanThreads; each group of 256 threads sums a share of the
// workgroups, with independent loads in flight.
// ---------------------------------------------------------------------------
constexpr int kPlanThreads = 1024;

__global__ __launch_bounds__(kPlanThreads) void k_tile_plan(const uint32_t* __restrict__ part, uint32_t groups,
                                                            int digits, uint64_t n, uint64_t* hist,
                                                            uint64_t* base, uint32_t* plan, bool clobber,
                                                            int trie_bits) {
    constexpr int Q = kPlanThreads / kRadix;
    __shared__ uint64_t s_h[Q][kRadix];
    const int tid = threadIdx.x, b = tid % kRadix, q = tid / kRadix;
    uint64_t h[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int j = 0; j < digits; ++j) {
        uint64_t acc = 0;
        constexpr int kBatch = 8;
        for (uint32_t g0 = q; g0 < groups; g0 += Q * kBatch) {
            uint32_t v[kBatch];
#pragma unroll
            for (int i = 0; i < kBatch; ++i) {
                const uint32_t g = g0 + i * Q;
                v[i] = g < groups ? part[((uint64_t)g * digits + j) * kRadix + b] : 0u;
            }
#pragma unroll
            for (int i = 0; i < kBatch; ++i) acc += v[i];
        }
        s_h[q][b] = acc;
        __syncthreads();
        if (q == 0) {
#pragma unroll
            for (int i = 1; i < Q; ++i) acc += s_h[i][b];
            h[j] = acc;
        }
        __syncthreads();
    }
    finish_plan(h, digits, n, hist, base, plan, clobber, trie_bits);
}

hipError_t launch_tile_plan(const uint32_t* part, uint32_t groups, int digits, uint64_t n, uint64_t* hist,
                            uint64_t* base, uint32_t* plan, hipStream_t s, bool clobber, int trie_bits) {
    k_tile_plan<<<1, kPlanThreads, 0, s>>>(part, groups, digits, n, hist, base, plan, clobber, trie_bits);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Step 2: the other two offset levels.  A super-block is 256 blocks, so its
// prefixes stay below 2^24.
//   bsum[b][d]  <- counts of d in the blocks of b's super-block before b
//                  (in place); ssum[s][d] <- super-block total
//   sbase[s][d] <- start of d in the pass output + counts of d in all
//                  super-blocks before s
// The output position of tile t's first key of digit d is then
//   sbase[s][d] + bsum[b][d] + th[t][d].
// One thread per digit value; loads are batched so the in-place update does
// not serialise them.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kRadix) void k_block_rel(TiledArgs a, int pass) {
    if (!a.plan[4 * pass]) return;
    const uint64_t sb = blockIdx.x;
    const uint32_t d = threadIdx.x;
    const uint64_t blocks = (a.tiles + a.block_tiles - 1) / a.block_tiles;
    const uint64_t b0 = sb * kSuperBlock;
    const uint64_t b1 = b0 + kSuperBlock < blocks ? b0 + kSuperBlock : blocks;
    constexpr int kBatch = 64;  // loads in flight per round trip
    uint32_t run = 0;
    for (uint64_t b = b0; b < b1; b += kBatch) {
        uint32_t c[kBatch];
#pragma unroll
        for (int i = 0; i < kBatch; ++i) {
            // clamped index: every load is issued unconditionally, so the
            // whole batch is in flight at once; the clamped ones are unused
            const uint64_t j = b + i < b1 ? b + i : b1 - 1;
            c[i] = a.bsum[j * kRadix + d];
        }
#pragma unroll
        for (int i = 0; i < kBatch; ++i) {
            if (b + i < b1) {
                a.bsum[(b + i) * kRadix + d] = run;
                run += c[i];
            }
        }
    }
    a.ssum[sb * kRadix + d] = run;
}

__global__ __launch_bounds__(kRadix) void k_super_base(TiledArgs a, int pass) {
    if (!a.plan[4 * pass]) return;
    const uint32_t d = threadIdx.x;
    const uint64_t blocks = (a.tiles + a.block_tiles - 1) / a.block_tiles;
    const uint64_t supers = (blocks + kSuperBlock - 1) / kSuperBlock;
    uint64_t run = a.base[(uint64_t)a.plan[4 * pass + 3] * 2 * kRadix + d];
    constexpr int kBatch = 32;  // loads in flight per round trip
    for (uint64_t sb0 = 0; sb0 < supers; sb0 += kBatch) {
        uint32_t c[kBatch];
#pragma unroll
        for (int i = 0; i < kBatch; ++i) {
            const uint64_t j = sb0 + i < supers ? sb0 + i : supers - 1;  // clamped, as above
            c[i] = a.ssum[j * kRadix + d];
        }
#pragma unroll
        for (int i = 0; i < kBatch; ++i) {
            if (sb0 + i < supers) {
                a.sbase[(sb0 + i) * kRadix + d] = run;
                run += c[i];
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Step 3: scatter.  Tile slot i (input order) of wave w, item k, lane l is
// i = w*64*ITEMS + k*64 + l, so a wave's items cover a contiguous stretch in
// input order and the per-wave ranks (wave_rank) are stable.
//
// The loop is software-pipelined: the next tile's keys, payloads, offsets
// and ticket are requested in this iteration and consumed at the top of the
// next one -- right after the first barrier, or with LATE only once this
// tile is staged, so that neither prefetch occupies registers while the
// tile is ranked (what lets a 16-item, 8192-key tile fit two workgroups per
// CU without spilling: longer per-digit runs, fewer partial lines).  The
// ticket is always taken after the first barrier.  Every global load and store in the loop is
// issued unconditionally (out-of-range lanes load a valid address and store
// to the workspace's sink word), so the number of memory operations between
// a request and its use is fixed and the wait at the top of the loop leaves
// the previous tile's stores in flight.
// ---------------------------------------------------------------------------
// What a pass writes of its keys: the keys (kOutKeys), nothing (kOutNone:
// the second pass of a 16-bit pair sort, whose sorted keys are expanded
// from the 2^16-bin histogram), or only their high bytes, to a.narrow
// (kOutHigh: the first pass of a 16-bit pair sort, for the second pass).
constexpr int kOutKeys = 0, kOutNone = 1, kOutHigh = 2;

template <typename K, typename V, int THREADS, int ITEMS, bool LATE, int KOUT, bool ORD>
__global__ __launch_bounds__(THREADS) __attribute__((amdgpu_waves_per_eu(4)))
void k_tile_scatter(TiledArgs a, int pass) {
    constexpr int W = THREADS / kWave;
    constexpr int T = THREADS * ITEMS;
    constexpr int VK = 16 / sizeof(K);
    constexpr int NV = T / VK + 1;                   // aligned vectors covering any tile
    constexpr int R = (NV + THREADS - 1) / THREADS;  // vectors per thread
    constexpr bool kHasVals = !std::is_same<V, NoVal>::value;
    using VS = typename std::conditional<kHasVals, V, uint32_t>::type;
    static_assert(THREADS >= kRadix, "one thread per digit value");
    static_assert(T < 65536, "tile counts are 16-bit");
    constexpr bool kLateVals = LATE;
    // wide keys with payloads on LATE (8192-key) tiles: the payloads are
    // fetched only once the tile's keys are staged in sorted order (their
    // registers are free then) and go through the key buffer after the keys
    // are stored, so the tile fits LDS twice per CU; the next tile's keys
    // are requested while the payloads are stored
    constexpr bool kSplit = kHasVals && LATE && sizeof(K) >= 4 && sizeof(VS) <= sizeof(K);

    __shared__ uint64_t s_peers[W][kRadix];
    __shared__ uint32_t s_wcnt[W][kRadix];
    __shared__ uint64_t s_dst[kRadix];  // output position of staged slot q is s_dst[d] + q
    __shared__ uint64_t s_wsum[4];
    __shared__ uint32_t s_next;
    __shared__ __attribute__((aligned(16))) K s_keys[NV * VK];  // slot T: sink of a bad rank
    // 64-bit keys: tiles holding at most kQuadDigits digit values (runs of
    // 1024 slots on average, as in presorted input) write four slots per
    // thread at a time, other tiles one (four-slot groups straddling a
    // digit boundary would make each wave run both paths).  The u64 passes
    // measured 2-6% faster with this code even where no tile takes it
    // (its tiles then hold every digit value): a code and LDS layout
    // effect.  Narrower keys measured slower with it (the headline u16
    // pairs 1.5%) and do without.
    constexpr bool kQuadOK = !kSplit && ITEMS % 4 == 0 && sizeof(K) == 8;
    constexpr uint32_t kQuadDigits = 8;
    __shared__ __attribute__((aligned(kQuadOK ? 16 : alignof(VS)))) VS s_vals[kHasVals && !kSplit ? T + 1 : 1];
    __shared__ uint32_t s_nz[kQuadOK ? kRadix / kWave : 1];

    if (!a.plan[4 * pass]) return;
    const uint32_t src_sel = a.plan[4 * pass + 1], dst_sel = a.plan[4 * pass + 2];
    // the second pass of a 16-bit pair sort reads the high key bytes as
    // one-byte keys
    const bool narrow_src = sizeof(K) == 1 && a.narrow != nullptr;
    const K* src_k = narrow_src ? reinterpret_cast<const K*>(a.narrow) : pass_source<K>(a, src_sel);
    K* dst_k = static_cast<K*>(dst_sel == kBufOut ? a.out_k : a.tmp_k);
    const VS* src_v = nullptr;
    VS* dst_v = nullptr;
    if constexpr (kHasVals) {
        src_v = static_cast<const VS*>(src_sel == kBufIn ? a.in_v : src_sel == kBufOut ? a.out_v : a.tmp_v);
        dst_v = static_cast<VS*>(dst_sel == kBufOut ? a.out_v : a.tmp_v);
    }
    K* sink_k = reinterpret_cast<K*>(a.sink);
    VS* sink_v = reinterpret_cast<VS*>(a.sink);
    const int shift = sizeof(K) == 1 ? 0 : 8 * (int)a.plan[4 * pass + 3];  // one-byte keys: one digit
    // the high bytes matter only if the second pass runs
    const bool write_high = KOUT == kOutHigh && a.plan[4 * 1] != 0;
    uint8_t* sink_b = reinterpret_cast<uint8_t*>(a.sink);

    // contiguous tile group of this workgroup's XCD; its workgroups take the
    // group's tiles in order from a ticket counter, so the tiles in flight
    // on the XCD stay consecutive whatever the speed of each workgroup
    const uint32_t groups = (gridDim.x % kXcds == 0) ? kXcds : 1u;
    const uint32_t x = blockIdx.x % groups;
    const uint64_t tlo = a.tiles * x / groups, thi = a.tiles * (x + 1) / groups;
    // the counter's address is made opaque to the compiler so that the
    // ticket request stays a plain returning atomic whose result is waited
    // for where it is used, one tile later
    uint32_t opaque = 0;
    asm volatile("" : "+v"(opaque));
    uint32_t* ctr = a.tickets + ((uint64_t)pass * kXcds + x) * kTicketStride + opaque;

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    for (int i = tid; i < W * kRadix; i += THREADS) (&s_peers[0][0])[i] = 0;
    const uint32_t wbase = (uint32_t)wave * kWave * ITEMS;
    const uint32_t dig = (uint32_t)tid & (kRadix - 1);
    const uint16_t* th16 = reinterpret_cast<const uint16_t*>(a.th);
    const uint32_t head = (uint32_t)((reinterpret_cast<uintptr_t>(src_k) & 15) / sizeof(K));

    // tile t's keys [tb, tb + cnt) lie in the aligned vectors starting at
    // key index tb - sh, sh = (tb + head) mod VK
    u32x4 nkv[R];
    VS nval[ITEMS];
    uint64_t nsb = 0;
    uint32_t nbo = 0, nto = 0;
    auto fetch_keys = [&](uint64_t t) {
        const uint64_t tb = t * T;
        const uint32_t cnt = (uint32_t)((a.n - tb) < (uint64_t)T ? (a.n - tb) : T);
        const uint32_t sh = (uint32_t)((tb + head) % VK);
        const uint32_t nv = (sh + cnt + VK - 1) / VK;
        const u32x4* gv = reinterpret_cast<const u32x4*>(src_k + (tb - sh));
        const uint64_t b = t / a.block_tiles, sb = b / kSuperBlock;
        nsb = a.sbase[sb * kRadix + dig];
        nbo = a.bsum[b * kRadix + dig];
        nto = th16[t * kRadix + dig];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const uint32_t v = tid + r * THREADS;
            nkv[r] = __builtin_nontemporal_load(&gv[v < nv ? v : nv - 1]);
        }
    };
    auto fetch_vals = [&](uint64_t t) {
        if constexpr (kHasVals) {
            const uint64_t tb = t * T;
            const uint32_t cnt = (uint32_t)((a.n - tb) < (uint64_t)T ? (a.n - tb) : T);
#pragma unroll
            for (int k = 0; k < ITEMS; ++k) {
                const uint32_t idx = wbase + k * kWave + lane;
                nval[k] = __builtin_nontemporal_load(&src_v[tb + (idx < cnt ? idx : cnt - 1)]);
            }
        }
    };

    uint32_t ticket = 0;
    if (tid == 0) s_next = atomicAdd(ctr, 1u);
    __syncthreads();
    uint64_t t = tlo + s_next;
    bool bad_rank = false, bad_dst = false;
    if (t < thi) {
        if (tid == 0) ticket = atomicAdd(ctr, 1u);
        fetch_keys(t);
        if constexpr (!kSplit) fetch_vals(t);
        // drain the first requests here, so that at the top of the loop only
        // the previous tile's stores can be outstanding (vmcnt(0))
        __builtin_amdgcn_s_waitcnt(0x0F70);
        __syncthreads();  // s_next read by all before it is rewritten
        for (;;) {
            const uint64_t tb = t * T;
            const uint32_t count = (uint32_t)((a.n - tb) < (uint64_t)T ? (a.n - tb) : T);
            const uint32_t sh = (uint32_t)((tb + head) % VK);  // tile key i sits at s_keys[i + sh]
            const uint32_t nv = (sh + count + VK - 1) / VK;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const uint32_t v = tid + r * THREADS;
                // ranks and digits refer to the mapped key (order_map)
                if (v < nv)
                    reinterpret_cast<u32x4*>(s_keys)[v] = ORD ? order_map_vec<K>(nkv[r], a.ord_pos, a.ord_neg) : nkv[r];
            }
            // payloads of this tile: copied out of the prefetch registers,
            // or (kLateVals) used from them directly, the next tile's keys
            // and payloads being requested only after staging
            VS val[ITEMS];
            if constexpr (kHasVals && !kLateVals) {
#pragma unroll
                for (int k = 0; k < ITEMS; ++k) val[k] = nval[k];
            }
            const uint64_t off = nsb + nbo + nto;
            if (tid == 0) s_next = ticket;
#pragma unroll
            for (int i = 0; i < kRadix / kWave; ++i) s_wcnt[wave][lane + kWave * i] = 0;
            __syncthreads();
            const uint64_t tn = tlo + s_next;
            const bool more = tn < thi;
            if (tid == 0) ticket = atomicAdd(ctr, 1u);
            // the last fetch repeats this tile and is not used
            if constexpr (!kLateVals) {
                fetch_keys(more ? tn : t);
                fetch_vals(more ? tn : t);
            }

            // keys of up to 16 bits share a register with their rank (rank < T < 2^16)
            constexpr bool kPack = sizeof(K) <= 2;
            K key[kPack ? 1 : ITEMS];
            uint32_t kr[ITEMS];  // kPack: key | rank << 16; otherwise the rank
#pragma unroll
            for (int k = 0; k < ITEMS; ++k) {
                const uint32_t idx = wbase + k * kWave + lane;
                const K kk = idx < count ? s_keys[idx + sh] : (K)0;
                if constexpr (kPack) kr[k] = kk;
                else key[k] = kk;
            }
            // a full tile (every tile but the last) ranks without lane masks
            const bool full = count == (uint32_t)T;
            auto rank_items = [&](auto full_c) {
                constexpr bool FULL = decltype(full_c)::value;
#pragma unroll
                for (int k = 0; k < ITEMS; ++k) {
                    const bool valid = FULL || wbase + k * kWave + lane < count;
                    const K kk = kPack ? (K)kr[k] : key[kPack ? 0 : k];
                    const uint32_t r =
                        wave_rank_uniform_first<FULL>(digit_of<K>(kk, shift), valid, s_peers[wave], s_wcnt[wave]);
                    if constexpr (kPack) kr[k] |= r << 16;
                    else kr[k] = r;
                }
            };
            if (full) rank_items(std::true_type{});
            else rank_items(std::false_type{});
            __syncthreads();

            // tile histogram from the wave counts, its exclusive scan, and
            // the per-wave bases of every digit
            uint32_t h = 0;
            if (tid < kRadix) {
#pragma unroll
                for (int w = 0; w < W; ++w) h += s_wcnt[w][tid];
            }
            uint64_t total;
            const uint32_t start = (uint32_t)scan256_exclusive<uint64_t>(tid < kRadix ? h : 0, s_wsum, &total);
            if (tid < kRadix) {
                uint32_t run = start;
#pragma unroll
                for (int w = 0; w < W; ++w) {
                    const uint32_t c = s_wcnt[w][tid];
                    s_wcnt[w][tid] = run;
                    run += c;
                }
                s_dst[tid] = off - start;
            }
            if constexpr (kQuadOK) {  // digit values present in the tile
                const uint64_t nzm = ballot(tid < kRadix && h != 0);
                if (lane == 0 && tid < kRadix) s_nz[wave] = popc64(nzm);
            }
            __syncthreads();
            bool few_runs = false;
            if constexpr (kQuadOK) {
                uint32_t nz = 0;
#pragma unroll
                for (int i = 0; i < kRadix / kWave; ++i) nz += s_nz[i];
                few_runs = nz <= kQuadDigits;
            }

#pragma unroll
            for (int k = 0; k < ITEMS; ++k) {
                if (wbase + k * kWave + lane < count) {
                    const K kk = kPack ? (K)(kr[k] & 0xFFFFu) : key[kPack ? 0 : k];
                    const uint32_t r = kPack ? kr[k] >> 16 : kr[k];
                    const uint32_t pos = s_wcnt[wave][digit_of<K>(kk, shift)] + r;
                    bad_rank |= pos >= (uint32_t)T;
                    const uint32_t p = pos < (uint32_t)T ? pos : (uint32_t)T;
                    s_keys[p] = kk;
                    if constexpr (kSplit) kr[k] = p;  // the payload's slot
                    else if constexpr (kHasVals) s_vals[p] = kLateVals ? nval[k] : val[k];
                }
            }
            if constexpr (kSplit) {
                __builtin_amdgcn_sched_barrier(0);  // not above the key staging
                fetch_vals(t);  // this tile's payloads, staged after its keys are stored
            } else if constexpr (kLateVals) {
                fetch_keys(more ? tn : t);
                fetch_vals(more ? tn : t);
            }
            __syncthreads();

            uint32_t dg[kSplit ? (ITEMS + 3) / 4 : 1];  // digits of this thread's slots (split staging)
            if constexpr (kQuadOK) {
                if (few_runs) {
                    // slots 4i..4i+3: their keys in one LDS read; when all
                    // four are in the tile and share a digit (one run of the
                    // output; staged slots are in digit order), one
                    // destination lookup, their payloads in one read, and
                    // one store each of keys and payloads
                    typedef VS vs4 __attribute__((ext_vector_type(4), aligned(sizeof(VS))));
                    typedef K k4 __attribute__((ext_vector_type(4), aligned(sizeof(K))));
                    auto write_slot = [&](uint32_t q) {
                        const bool in = q < count;
                        const uint32_t qq = in ? q : 0u;
                        const K kk = s_keys[qq];
                        const uint64_t dst = s_dst[digit_of<K>(kk, shift)] + qq;
                        const bool ok = in && dst < a.n;
                        bad_dst |= in && !(dst < a.n);
                        if constexpr (KOUT == kOutKeys)
                            *(ok ? dst_k + dst : sink_k) = ORD ? order_unmap<K>(kk, (K)a.ord_pos, (K)a.ord_neg) : kk;
                        if constexpr (kHasVals) *(ok ? dst_v + dst : sink_v) = s_vals[qq];
                    };
#pragma unroll
                    for (int k = 0; k < ITEMS / 4; ++k) {
                        const uint32_t q0 = 4u * (k * THREADS + tid);  // at most T - 4
                        K kq[4];
                        __builtin_memcpy(kq, &s_keys[q0], 4 * sizeof(K));
                        const uint32_t d0 = digit_of<K>(kq[0], shift);
                        if (q0 + 4 <= count && d0 == digit_of<K>(kq[3], shift)) {
                            const uint64_t dst = s_dst[d0] + q0;
                            const bool ok = dst + 4 <= a.n;
                            bad_dst |= !ok;
                            if (ok) {
                                if constexpr (KOUT == kOutKeys) {
                                    k4 o;
#pragma unroll
                                    for (int j = 0; j < 4; ++j)
                                        o[j] = ORD ? order_unmap<K>(kq[j], (K)a.ord_pos, (K)a.ord_neg) : kq[j];
                                    *reinterpret_cast<k4*>(dst_k + dst) = o;
                                }
                                if constexpr (kHasVals)
                                    *reinterpret_cast<vs4*>(dst_v + dst) = *reinterpret_cast<const vs4*>(&s_vals[q0]);
                            }
                        } else {
#pragma unroll
                            for (int j = 0; j < 4; ++j) write_slot(q0 + j);
                        }
                        if (k & 1) __builtin_amdgcn_sched_barrier(0);
                    }
                }
            }
#pragma unroll
            for (int k = 0; k < ITEMS; ++k) {
                if (few_runs) break;  // tile-uniform: written four slots at a time above
                const uint32_t q = k * THREADS + tid;
                const bool in = q < count;
                const uint32_t qq = in ? q : 0u;
                const K kk = s_keys[qq];
                const uint64_t dst = s_dst[digit_of<K>(kk, shift)] + qq;
                const bool ok = in && dst < a.n;
                bad_dst |= in && !(dst < a.n);
                if constexpr (KOUT == kOutKeys)
                    *(ok ? dst_k + dst : sink_k) = ORD ? order_unmap<K>(kk, (K)a.ord_pos, (K)a.ord_neg) : kk;
                if constexpr (KOUT == kOutHigh) {  // the mapped key's high byte
                    if (write_high) *(ok ? a.narrow + dst : sink_b) = (uint8_t)((uint32_t)kk >> 8);
                }
                if constexpr (kSplit) {
                    if (k % 4 == 0) dg[k / 4] = 0;
                    dg[k / 4] |= digit_of<K>(kk, shift) << (8 * (k % 4));
                } else if constexpr (kHasVals) {
                    *(ok ? dst_v + dst : sink_v) = s_vals[qq];
                }
                // keep the compiler from hoisting every slot's loads at once
                // (a barrier every 8 slots measured 0.1-0.5% faster than
                // every 4 on 2^31-key sorts of 16- and 32-bit keys, every 2
                // slower; 64-bit keys measured 1% faster with every 4)
                constexpr int kSchedEvery = sizeof(K) == 8 ? 4 : 8;
                if (k % kSchedEvery == kSchedEvery - 1) __builtin_amdgcn_sched_barrier(0);
            }
            if constexpr (kSplit) {
                // the payloads, through the key buffer at their keys' slots
                VS* s_pv = reinterpret_cast<VS*>(s_keys);
                __syncthreads();
#pragma unroll
                for (int k = 0; k < ITEMS; ++k)
                    if (wbase + k * kWave + lane < count) s_pv[kr[k]] = nval[k];
                // the next tile's keys, in flight while the payloads are stored
                fetch_keys(more ? tn : t);
                __syncthreads();
#pragma unroll
                for (int k = 0; k < ITEMS; ++k) {
                    const uint32_t q = k * THREADS + tid;
                    const bool in = q < count;
                    const uint32_t qq = in ? q : 0u;
                    const uint64_t dst = s_dst[(dg[k / 4] >> (8 * (k % 4))) & 0xFFu] + qq;
                    const bool ok = in && dst < a.n;
                    *(ok ? dst_v + dst : sink_v) = s_pv[qq];
                    if ((k & 3) == 3) __builtin_amdgcn_sched_barrier(0);
                }
            }
            __syncthreads();
            if (!more) break;
            t = tn;
        }
    }
    if (bad_rank) atomicOr(a.err, 4u);
    if (bad_dst) atomicOr(a.err, 8u);
}

// ---------------------------------------------------------------------------
// Sparse-trie fixup (Algorithm 5: the bins of the trie in order, each bin's
// entries ordered by their trailing bits).  The window passes have left the
// keys stably sorted by their bits from `shift` up, so every bin is a run of
// consecutive keys; runs are short when n is far below 2^p.  Each run is
// sorted by the whole key (its high bits are equal) by the thread at its
// first position, with a stable insertion sort, payloads moving alongside.
// A workgroup loads a tile of kTrieTile keys (and payloads) with the key
// before it and kTrieRun keys after it into LDS, finds the runs that start
// in the tile there and sorts the ones out of order in LDS.  If it sorted
// any, it writes back the slots it owns -- from its first run start to the
// end of the run holding its last position -- in one coalesced pass.  A run
// longer than kTrieRun keys is listed instead (its first
// position) for k_trie_longruns; a full list switches on the fallback.
// Runs are disjoint and found from their high bits only, which no sort
// changes, and each position is written only by the workgroup whose tile
// holds the first position of its run, so nothing races.
// ---------------------------------------------------------------------------
constexpr uint32_t kTrieRun = 64;
constexpr uint32_t kTrieLdsRun = 4096;
constexpr uint32_t kTrieTile = 2048;
constexpr int kTrieThreads = 256;

template <typename K>
__device__ __forceinline__ void trie_fallback(const TiledArgs& a) {
    // switch on the fallback slots and their copy word (the same words from
    // every caller)
    uint32_t* plan = const_cast<uint32_t*>(a.plan);
    for (int sl = kPlanCondSlot; sl < kPlanSlots; ++sl)
        if (plan[4 * sl + 1] != plan[4 * sl + 2])
            __hip_atomic_store(&plan[4 * sl], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(&plan[kPlanCopyTmp], plan[kPlanCondCopyTmp], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <typename K, typename V, bool ORD>
__global__ __launch_bounds__(kTrieThreads) void k_trie_fixup(TiledArgs a) {
    constexpr bool kHasVals = !std::is_same<V, NoVal>::value;
    using VS = typename std::conditional<kHasVals, V, uint32_t>::type;
    // a tile of kTrieTile positions, the key before it and kTrieRun keys
    // after it (a run that starts in the tile ends within them or is long)
    constexpr uint32_t kSpan = kTrieTile + kTrieRun + 1;
    __shared__ K s_key[kSpan];
    __shared__ VS s_val[kHasVals ? kSpan : 1];
    if (!a.plan[kPlanTrie]) return;
    const uint32_t buf = a.plan[kPlanFixBuf];
    K* keys = static_cast<K*>(buf == kBufOut ? a.out_k : a.tmp_k);
    VS* vals = nullptr;
    if constexpr (kHasVals) vals = static_cast<VS*>(buf == kBufOut ? a.out_v : a.tmp_v);
    const int shift = (int)a.plan[kPlanTrieShift];
    const K pos = (K)a.ord_pos, neg = (K)a.ord_neg;
    auto high = [&](K m) -> uint64_t { return (uint64_t)m >> shift; };
    const uint64_t n = a.n;
    const uint64_t tiles = (n + kTrieTile - 1) / kTrieTile;
    const int tid = threadIdx.x;
    bool overflow = false;
    // the span of tile t: positions [lo, hi) into slots [off, off + hi - lo)
    // (slot q holds position t0 - 1 + q); its keys and payloads are loaded
    // into registers one tile ahead, every load issued at a clamped index
    constexpr int kLoads = (kSpan + kTrieThreads - 1) / kTrieThreads;
    K rk[kLoads];
    VS rv[kLoads];
    auto span = [&](uint64_t t, uint64_t* lo, uint64_t* hi, uint32_t* off) {
        const uint64_t t0 = t * kTrieTile;
        *lo = t0 ? t0 - 1 : 0;
        *hi = t0 + kTrieTile + kTrieRun < n ? t0 + kTrieTile + kTrieRun : n;
        *off = t0 ? 0u : 1u;  // tile 0 has no key before it
    };
    auto fetch = [&](uint64_t t) {
        uint64_t lo, hi;
        uint32_t off;
        span(t, &lo, &hi, &off);
#pragma unroll
        for (int k = 0; k < kLoads; ++k) {
            const uint64_t p = lo + tid + (uint64_t)k * kTrieThreads;
            const uint64_t pc = p < hi ? p : hi - 1;
            rk[k] = keys[pc];
            if constexpr (kHasVals) rv[k] = vals[pc];
        }
    };
    if ((uint64_t)blockIdx.x < tiles) fetch(blockIdx.x);
    for (uint64_t t = blockIdx.x; t < tiles; t += gridDim.x) {
        const uint64_t t0 = t * kTrieTile;
        uint64_t lo, hi;
        uint32_t off;
        span(t, &lo, &hi, &off);
#pragma unroll
        for (int k = 0; k < kLoads; ++k) {
            const uint64_t p = lo + tid + (uint64_t)k * kTrieThreads;
            if (p < hi) {
                s_key[p - lo + off] = ORD ? order_map<K>(rk[k], pos, neg) : rk[k];
                if constexpr (kHasVals) s_val[p - lo + off] = rv[k];
            }
        }
        __syncthreads();
        if (t + gridDim.x < tiles) fetch(t + gridDim.x);  // in flight while this tile is worked on
        const uint32_t have = (uint32_t)(hi - lo) + off;  // slots filled: [off, have)
        // every loaded slot from the tile's first position on: the slots of
        // runs that start in the tile (slots 1..kTrieTile), including their
        // ends past it, are this tile's to place
        for (uint32_t q = 1 + tid; q < have; q += kTrieThreads) {
            const K kq = s_key[q];
            const uint64_t h = high(kq);
            uint32_t b = q;  // the run's first slot (or kTrieRun back)
            while (b > off && q - b < kTrieRun && high(s_key[b - 1]) == h) --b;
            if (b == 0 || b > kTrieTile) continue;  // a run of the tile before or after
            if (q - b >= kTrieRun) continue;        // inside a long run
            uint32_t e = q + 1;
            while (e < have && e - b <= kTrieRun && high(s_key[e]) == h) ++e;
            if (e - b > kTrieRun) {
                // a long run: listed by its first key, placed by k_trie_longruns
                if (q == b) {
                    const uint32_t slot = atomicAdd(a.trie_count, 1u);
                    if (slot < kTrieLongMax) a.trie_list[slot] = t0 + b - 1;
                    else overflow = true;
                }
                continue;
            }
            // rank in the run: keys that sort before this one (smaller, or
            // equal and earlier: stable)
            uint32_t rank = 0;
            for (uint32_t r = b; r < e; ++r) {
                const K kr = s_key[r];
                rank += (kr < kq || (kr == kq && r < q)) ? 1u : 0u;
            }
            const uint32_t dst = b + rank;
            if (dst != q) {
                keys[t0 + dst - 1] = ORD ? order_unmap<K>(kq, pos, neg) : kq;
                if constexpr (kHasVals) vals[t0 + dst - 1] = s_val[q];
            }
        }
        __syncthreads();
    }
    if (overflow) trie_fallback<K>(a);
}

// ---------------------------------------------------------------------------
// Long trie runs: one workgroup per listed run finds the run's end and
// whether it is in order, 256 keys at a time.  A run out of order of at most
// kTrieLdsRun keys is loaded into LDS and sorted there by a bitonic network
// over (mapped key, position in the run) -- positions are distinct, so the
// order is total and equal keys keep theirs (stable) -- then written back
// with its payloads.  A longer run out of order switches on the fallback.
// ---------------------------------------------------------------------------
template <typename K, typename V, bool ORD>
__global__ __launch_bounds__(kTrieThreads) void k_trie_longruns(TiledArgs a) {
    constexpr bool kHasVals = !std::is_same<V, NoVal>::value;
    using VS = typename std::conditional<kHasVals, V, uint32_t>::type;
    __shared__ K s_key[kTrieLdsRun];
    __shared__ VS s_val[kHasVals ? kTrieLdsRun : 1];
    __shared__ uint16_t s_idx[kTrieLdsRun];
    __shared__ uint64_t s_end;
    __shared__ int s_unordered;
    if (!a.plan[kPlanTrie]) return;
    const uint32_t listed = *a.trie_count;
    const uint32_t runs = listed < kTrieLongMax ? listed : kTrieLongMax;
    if (blockIdx.x >= runs) return;
    const uint32_t buf = a.plan[kPlanFixBuf];
    K* keys = static_cast<K*>(buf == kBufOut ? a.out_k : a.tmp_k);
    VS* vals = nullptr;
    if constexpr (kHasVals) vals = static_cast<VS*>(buf == kBufOut ? a.out_v : a.tmp_v);
    const int shift = (int)a.plan[kPlanTrieShift];
    const K pos = (K)a.ord_pos, neg = (K)a.ord_neg;
    auto mk = [&](uint64_t i) -> K { return ORD ? order_map<K>(keys[i], pos, neg) : keys[i]; };
    const uint64_t n = a.n;
    const int tid = threadIdx.x;
    for (uint32_t r = blockIdx.x; r < runs; r += gridDim.x) {
        const uint64_t b = a.trie_list[r];
        const uint64_t h = (uint64_t)mk(b) >> shift;
        if (tid == 0) {
            s_end = n;
            s_unordered = 0;
        }
        __syncthreads();
        // extent and order, 256 positions per step: the run ends at the
        // first position past it (or n); a step that holds it is the last
        for (uint64_t c = b;; c += kTrieThreads) {
            const uint64_t p = c + tid;
            bool stop = p >= n;
            if (!stop) {
                const K kp = mk(p);
                stop = ((uint64_t)kp >> shift) != h;
                if (!stop && p > b && kp < mk(p - 1)) s_unordered = 1;
            }
            if (stop) atomicMin(reinterpret_cast<unsigned long long*>(&s_end), (unsigned long long)p);
            __syncthreads();
            const uint64_t end_now = s_end;
            __syncthreads();  // every thread has read it before the next step may lower it
            if (end_now < c + kTrieThreads) break;
        }
        const uint64_t e = s_end;
        const int unordered = s_unordered;
        __syncthreads();
        if (!unordered) continue;
        const uint64_t len = e - b;
        if (len > kTrieLdsRun) {
            if (tid == 0) trie_fallback<K>(a);
            continue;
        }
        // load (mapped keys), bitonic sort of positions, write back
        uint32_t np2 = 1;
        while (np2 < len) np2 <<= 1;
        for (uint32_t i = tid; i < np2; i += kTrieThreads) {
            if (i < len) {
                s_key[i] = mk(b + i);
                if constexpr (kHasVals) s_val[i] = vals[b + i];
            }
            s_idx[i] = (uint16_t)i;
        }
        __syncthreads();
        auto before = [&](uint32_t x, uint32_t y) {
            // a strict total order: the run's keys by (key, position), then
            // the padding past the run by position
            const bool xp = x >= len, yp = y >= len;
            if (xp || yp) return xp && yp ? x < y : yp;
            return s_key[x] < s_key[y] || (s_key[x] == s_key[y] && x < y);
        };
        for (uint32_t k = 2; k <= np2; k <<= 1) {
            for (uint32_t jj = k >> 1; jj > 0; jj >>= 1) {
                for (uint32_t i = tid; i < np2; i += kTrieThreads) {
                    const uint32_t l = i ^ jj;
                    if (l > i) {
                        const uint32_t x = s_idx[i], y = s_idx[l];
                        const bool asc = (i & k) == 0;
                        if (asc ? before(y, x) : before(x, y)) {
                            s_idx[i] = (uint16_t)y;
                            s_idx[l] = (uint16_t)x;
                        }
                    }
                }
                __syncthreads();
            }
        }
        for (uint32_t i = tid; i < len; i += kTrieThreads) {
            const uint32_t x = s_idx[i];
            keys[b + i] = ORD ? order_unmap<K>(s_key[x], pos, neg) : s_key[x];
            if constexpr (kHasVals) vals[b + i] = s_val[x];
        }
        __syncthreads();
    }
}

template <typename K, typename V>
static void launch_fixup_kv(const TiledArgs& a, hipStream_t s) {
    const uint64_t tiles = (a.n + kTrieTile - 1) / kTrieTile;
    const uint32_t grid = (uint32_t)(tiles < 4096 ? (tiles ? tiles : 1) : 4096);
    if (a.ord_pos | a.ord_neg) k_trie_fixup<K, V, true><<<grid, kTrieThreads, 0, s>>>(a);
    else k_trie_fixup<K, V, false><<<grid, kTrieThreads, 0, s>>>(a);
}

template <typename K, typename V>
static void launch_longruns_kv(const TiledArgs& a, hipStream_t s) {
    const uint32_t grid = 512;
    if (a.ord_pos | a.ord_neg) k_trie_longruns<K, V, true><<<grid, kTrieThreads, 0, s>>>(a);
    else k_trie_longruns<K, V, false><<<grid, kTrieThreads, 0, s>>>(a);
}

hipError_t launch_trie_longruns(const TiledArgs& a, int key_bytes, int val_bytes, hipStream_t s) {
    if (key_bytes == 4) {
        if (val_bytes == 0) launch_longruns_kv<uint32_t, NoVal>(a, s);
        else if (val_bytes == 4) launch_longruns_kv<uint32_t, uint32_t>(a, s);
        else launch_longruns_kv<uint32_t, uint64_t>(a, s);
    } else if (key_bytes == 8) {
        if (val_bytes == 0) launch_longruns_kv<uint64_t, NoVal>(a, s);
        else if (val_bytes == 4) launch_longruns_kv<uint64_t, uint32_t>(a, s);
        else launch_longruns_kv<uint64_t, uint64_t>(a, s);
    } else {
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_trie_fixup(const TiledArgs& a, int key_bytes, int val_bytes, hipStream_t s) {
    if (key_bytes == 4) {
        if (val_bytes == 0) launch_fixup_kv<uint32_t, NoVal>(a, s);
        else if (val_bytes == 4) launch_fixup_kv<uint32_t, uint32_t>(a, s);
        else launch_fixup_kv<uint32_t, uint64_t>(a, s);
    } else if (key_bytes == 8) {
        if (val_bytes == 0) launch_fixup_kv<uint64_t, NoVal>(a, s);
        else if (val_bytes == 4) launch_fixup_kv<uint64_t, uint32_t>(a, s);
        else launch_fixup_kv<uint64_t, uint64_t>(a, s);
    } else {
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Tile shapes and launchers
// ---------------------------------------------------------------------------
#define FS_TILED_SHAPES(X)                 \
    X(uint8_t, NoVal, 512, 8, false)       \
    X(uint8_t, uint32_t, 512, 8, false)    \
    X(uint8_t, uint64_t, 512, 8, false)    \
    X(uint16_t, uint32_t, 512, 16, true)   \
    X(uint16_t, uint64_t, 512, 8, false)   \
    X(uint32_t, NoVal, 512, 16, true)      \
    X(uint32_t, uint32_t, 512, 16, true)   \
    X(uint32_t, uint64_t, 512, 8, false)   \
    X(uint64_t, NoVal, 512, 8, false)      \
    X(uint64_t, uint32_t, 512, 8, false)   \
    X(uint64_t, uint64_t, 512, 4, false)

template <typename V>
constexpr int val_size() {
    if constexpr (std::is_same<V, NoVal>::value) return 0;
    else return (int)sizeof(V);
}

ScatterShape tiled_shape(int key_bytes, int val_bytes) {
#define FS_SHAPE(K, V, THR, IT, LATE) \
    if (key_bytes == (int)sizeof(K) && val_bytes == val_size<V>()) return ScatterShape{THR, IT};
    FS_TILED_SHAPES(FS_SHAPE)
#undef FS_SHAPE
    return ScatterShape{0, 0};
}

int tiled_scatter_per_cu(int key_bytes, int val_bytes) {
    int per_cu = 0;
    hipError_t e = hipErrorInvalidValue;
#define FS_OCC(K, V, THR, IT, LATE)                                                                  \
    if (key_bytes == (int)sizeof(K) && val_bytes == val_size<V>())                                   \
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_tile_scatter<K, V, THR, IT, LATE, kOutKeys, false>, THR, 0);
    FS_TILED_SHAPES(FS_OCC)
#undef FS_OCC
    return (e == hipSuccess && per_cu > 0) ? per_cu : 1;
}

template <typename K, int TILE, bool ORD>
static void launch_hist_o(const TiledArgs& a, int pass, bool first, uint32_t groups, hipStream_t s) {
    if (first) k_tile_hist<K, true, TILE, ORD><<<groups, kTileHistThreads, 0, s>>>(a, pass);
    else k_tile_hist<K, false, TILE, ORD><<<groups, kTileHistThreads, 0, s>>>(a, pass);
}

template <typename K, int TILE>
static void launch_hist_t(const TiledArgs& a, int pass, bool first, uint32_t groups, hipStream_t s) {
    if (a.ord_pos | a.ord_neg) launch_hist_o<K, TILE, true>(a, pass, first, groups, s);
    else launch_hist_o<K, TILE, false>(a, pass, first, groups, s);
}

hipError_t launch_tile_hist(const TiledArgs& a, int key_bytes, int pass, uint32_t groups, hipStream_t s,
                            bool first) {
    if (key_bytes == 1 && a.tile == 4096) launch_hist_t<uint8_t, 4096>(a, pass, first, groups, s);
    else if (key_bytes == 1 && a.tile == 8192) launch_hist_t<uint8_t, 8192>(a, pass, first, groups, s);
    else if (key_bytes == 2 && a.tile == 4096) launch_hist_t<uint16_t, 4096>(a, pass, first, groups, s);
    else if (key_bytes == 2 && a.tile == 8192) launch_hist_t<uint16_t, 8192>(a, pass, first, groups, s);
    else if (key_bytes == 2 && a.tile == 16384) launch_hist_t<uint16_t, 16384>(a, pass, first, groups, s);
    else if (key_bytes == 4 && a.tile == 4096) launch_hist_t<uint32_t, 4096>(a, pass, first, groups, s);
    else if (key_bytes == 4 && a.tile == 8192) launch_hist_t<uint32_t, 8192>(a, pass, first, groups, s);
    else if (key_bytes == 4 && a.tile == 2048) launch_hist_t<uint32_t, 2048>(a, pass, first, groups, s);
    else if (key_bytes == 8 && a.tile == 4096) launch_hist_t<uint64_t, 4096>(a, pass, first, groups, s);
    else if (key_bytes == 8 && a.tile == 2048) launch_hist_t<uint64_t, 2048>(a, pass, first, groups, s);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_tile_offsets(const TiledArgs& a, int pass, hipStream_t s) {
    const uint64_t blocks = (a.tiles + a.block_tiles - 1) / a.block_tiles;
    const uint64_t supers = (blocks + kSuperBlock - 1) / kSuperBlock;
    k_block_rel<<<(uint32_t)supers, kRadix, 0, s>>>(a, pass);
    k_super_base<<<1, kRadix, 0, s>>>(a, pass);
    return hipGetLastError();
}

// 16-bit keys are tiled only in pair sorts, whose first pass writes the
// high key bytes (kOutHigh); every other width writes its keys
template <typename K, typename V, int THR, int IT, bool LATE>
static hipError_t scatter_launch(const TiledArgs& a, int pass, uint32_t groups, hipStream_t s) {
    constexpr int kout = (sizeof(K) == 2 && !std::is_same<V, NoVal>::value) ? kOutHigh : kOutKeys;
    if (a.ord_pos | a.ord_neg) k_tile_scatter<K, V, THR, IT, LATE, kout, true><<<groups, THR, 0, s>>>(a, pass);
    else k_tile_scatter<K, V, THR, IT, LATE, kout, false><<<groups, THR, 0, s>>>(a, pass);
    return hipGetLastError();
}

hipError_t launch_tile_scatter(const TiledArgs& a, int key_bytes, int val_bytes, int pass, uint32_t groups,
                               hipStream_t s) {
#define FS_LAUNCH_SHAPE(K, V, THR, IT, LATE)                                         \
    if (key_bytes == (int)sizeof(K) && val_bytes == val_size<V>())                   \
        return scatter_launch<K, V, THR, IT, LATE>(a, pass, groups, s);
    FS_TILED_SHAPES(FS_LAUNCH_SHAPE)
#undef FS_LAUNCH_SHAPE
    return hipErrorInvalidValue;
}

// the second pass of a 16-bit pair sort: one-byte keys (already mapped)
// on the 16-bit pair shape's tiles
template <typename K, typename V, int THR, int IT, bool LATE>
static hipError_t scatter_narrow_launch(const TiledArgs& a, int pass, uint32_t groups, hipStream_t s) {
    if constexpr (sizeof(K) == 2 && !std::is_same<V, NoVal>::value) {
        k_tile_scatter<uint8_t, V, THR, IT, LATE, kOutNone, false><<<groups, THR, 0, s>>>(a, pass);
        return hipGetLastError();
    }
    return hipErrorInvalidValue;
}

hipError_t launch_tile_scatter_narrow(const TiledArgs& a, int val_bytes, int pass, uint32_t groups,
                                      hipStream_t s) {
    if (!a.narrow) return hipErrorInvalidValue;
#define FS_LAUNCH_NARROW(K, V, THR, IT, LATE)                                        \
    if (sizeof(K) == 2 && val_bytes == val_size<V>() && val_bytes != 0)              \
        return scatter_narrow_launch<K, V, THR, IT, LATE>(a, pass, groups, s);
    FS_TILED_SHAPES(FS_LAUNCH_NARROW)
#undef FS_LAUNCH_NARROW
    return hipErrorInvalidValue;
}

// High bytes of the (mapped) input keys of a 16-bit pair sort whose first
// pass is skipped (every key has the same low byte) while the second runs.
__global__ void k_narrow_copy(TiledArgs a) {
    if (a.plan[0] || !a.plan[4]) return;
    const uint16_t* in = static_cast<const uint16_t*>(a.in_k);
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < a.n; i += stride) {
        uint16_t k = in[i];
        if (a.ord_pos | a.ord_neg) k = order_map<uint16_t>(k, (uint16_t)a.ord_pos, (uint16_t)a.ord_neg);
        a.narrow[i] = (uint8_t)(k >> 8);
    }
}

hipError_t launch_narrow_copy(const TiledArgs& a, hipStream_t s) {
    if (!a.narrow || a.n == 0) return hipErrorInvalidValue;
    uint64_t g = (a.n + 255) / 256;
    if (g > 8192) g = 8192;
    k_narrow_copy<<<(unsigned)g, 256, 0, s>>>(a);
    return hipGetLastError();
}

}  // namespace fs
