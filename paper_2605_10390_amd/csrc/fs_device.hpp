// Device-side helpers shared by the sort kernels (gfx950, wave64).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fs {

constexpr int kWave = 64;
constexpr int kRadixBits = 8;
constexpr int kRadix = 1 << kRadixBits;

// Bound on look-back polls before a workgroup gives up and raises the
// workspace error word (never reached by a correct launch; it keeps every
// wave finite).
constexpr uint32_t kSpinLimit = 1u << 26;

// Plan words written by the planning kernel and read by every pass kernel.
// Pass slot j (0..15): plan[4j] = active, plan[4j+1] = source buffer,
// plan[4j+2] = destination, plan[4j+3] = the 8-bit digit it sorts on.
// plan[kPlanCopy] = 1: the result is the input itself (no pass active, or
// an even number of clobbering passes), copied from keys_in to the output;
// plan[kPlanCopyTmp] = 1: the result sits in the temporary buffer.
// Trie plans (sparse keys, n far below 2^p): slots 0..7 sort the window
// digits, the fixup kernel sorts each run of equal window prefix in buffer
// plan[kPlanFixBuf] by the trailing bits below plan[kPlanTrieShift], and
// slots 8..15 hold a full LSD over every active digit that the fixup turns
// on (with plan[kPlanCondCopyTmp] as its copy word) only if some run is too
// long for it.  plan[kPlanRecount0] = 1: slot 0 sorts a digit other than 0,
// so its tile counts are taken again (the first read counts digit 0).
constexpr int kPlanSlots = 16;
constexpr int kPlanCondSlot = 8;
constexpr int kPlanCopy = 64;
constexpr int kPlanCopyTmp = 65;
constexpr int kPlanTrie = 66;
constexpr int kPlanTrieShift = 67;
constexpr int kPlanFixBuf = 68;
constexpr int kPlanCondCopyTmp = 69;
constexpr int kPlanRecount0 = 70;
constexpr int kPlanWords = 72;
enum BufSel : uint32_t { kBufIn = 0, kBufOut = 1, kBufTmp = 2 };

struct NoVal {};

// 16-byte vector usable with the non-temporal load/store builtins
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// A pointer known to address global memory.  Pointers read from memory
// (segment descriptors) are generic to the compiler, which then emits flat
// instructions; flat accesses count against the LDS wait counter too, so
// every LDS wait would also wait for them.
template <typename T>
using gptr = __attribute__((address_space(1))) T*;
template <typename T>
__device__ __forceinline__ gptr<T> to_global(T* p) {
    return (gptr<T>)p;
}

__device__ __forceinline__ uint64_t ballot(bool p) { return __builtin_amdgcn_ballot_w64(p); }

// number of set bits of m in lanes below this lane
__device__ __forceinline__ uint32_t lanes_below(uint64_t m) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

__device__ __forceinline__ uint32_t popc64(uint64_t m) { return (uint32_t)__builtin_popcountll(m); }

// A wave-uniform value that the optimiser must treat as new on every loop
// iteration.  A tile's alignment shift is the same for every tile (tile
// bases are multiples of the vector width), and the compiler would
// otherwise hoist every per-element index derived from it out of the tile
// loop and hold them all in registers for the loop's length (about 100
// VGPRs in the one-byte histogram, which then ran one workgroup per CU).
// No instruction is emitted.
__device__ __forceinline__ uint32_t each_iteration(uint32_t x) {
    asm volatile("" : "+s"(x));
    return x;
}

__device__ __forceinline__ uint32_t ld_agent(const uint32_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_agent(uint32_t* p, uint32_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint32_t add_agent(uint32_t* p, uint32_t v) {
    return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <typename K>
__device__ __forceinline__ uint32_t digit_of(K key, int shift) {
    if constexpr (sizeof(K) <= 4)
        return __builtin_amdgcn_ubfe((uint32_t)key, (uint32_t)shift, kRadixBits);
    else
        return shift < 32 ? __builtin_amdgcn_ubfe((uint32_t)key, (uint32_t)shift, kRadixBits)
                          : __builtin_amdgcn_ubfe((uint32_t)(key >> 32), (uint32_t)(shift - 32), kRadixBits);
}

// Key order.  Signed, floating-point and descending sorts are unsigned
// ascending sorts of a mapped key t = k ^ (top bit of k ? neg : pos), whose
// unsigned order is the wanted order of k:
//   unsigned  pos = neg = 0            signed  pos = neg = sign bit
//   float     pos = sign bit, neg = all ones (IEEE 754 totalOrder: negative
//             values have their magnitude bits reversed)
//   descending: both masks complemented.
// Kernels map keys where they load them and unmap them where they store
// them, so memory only ever holds the caller's key bits; digits, counts and
// ranks all refer to the mapped key.
template <typename K>
__device__ __forceinline__ K order_map(K k, K pos, K neg) {
    return k ^ ((k >> (8 * sizeof(K) - 1)) ? neg : pos);
}
// the inverse: the mask applied was `neg` exactly when undoing it leaves
// the top bit set
template <typename K>
__device__ __forceinline__ K order_unmap(K t, K pos, K neg) {
    return t ^ (((K)(t ^ neg) >> (8 * sizeof(K) - 1)) ? neg : pos);
}
// order_map of every key packed in a 16-byte vector
template <typename K>
__device__ __forceinline__ u32x4 order_map_vec(u32x4 q, uint64_t pos, uint64_t neg) {
    K k[16 / sizeof(K)];
    __builtin_memcpy(k, &q, 16);
#pragma unroll
    for (int e = 0; e < (int)(16 / sizeof(K)); ++e) k[e] = order_map<K>(k[e], (K)pos, (K)neg);
    __builtin_memcpy(&q, k, 16);
    return q;
}

// Compressed 2^16-bin histogram of 16-bit keys in LDS.
//
// Counter pair w holds bin 2w in its low half and bin 2w+1 in its high half.
// Every increment is a returning LDS add, so the adding lane sees the old
// word and can tell whether its add carried out of the low half (which also
// bumped the high half by one) or out of the whole word.  Atomic adds are
// linearised, so each wrap is seen by exactly one lane, which counts it in
// wrap_lo[w] or wrap_word[w] (global, rare: one per 65536 keys of a bin).
// Exact decode of the sums over all workgroups, with W_i the raw words:
//   lo  = sum(W_i & 0xFFFF) + 2^16 * wrap_lo[w]
//   V   = sum(W_i)          + 2^32 * wrap_word[w]     (= lo + 2^16 * hi)
//   hi  = (V - lo) / 2^16
__device__ __forceinline__ void hist16_add(uint32_t* cnt, uint32_t key, uint32_t c,
                                           uint32_t* wrap_lo, uint32_t* wrap_word) {
    const uint32_t w = key >> 1;
    const uint32_t inc = (key & 1u) ? (c << 16) : c;
    const uint32_t old = atomicAdd(&cnt[w], inc);
    const bool word_wrap = (old + inc) < old;
    const bool lo_wrap = ((old & 0xFFFFu) + (inc & 0xFFFFu)) > 0xFFFFu;
    if (__builtin_expect(word_wrap, 0)) atomicAdd(&wrap_word[w], 1u);
    if (__builtin_expect(lo_wrap, 0)) atomicAdd(&wrap_lo[w], 1u);
}

// Leader aggregation of one add per lane: the lanes whose bucket id equals
// that of the first active lane are summed into one add made by the lowest
// of them (the others add nothing).  For skewed keys the first lane's bucket
// is often a hot one, whose same-address adds would otherwise be serialised
// by the LDS; for spread keys it matches only itself and nothing changes.
// Lanes with in == false take no part.  Returns this lane's count; *shared
// (wave-uniform) is how many lanes held the leader's bucket.
__device__ __forceinline__ uint32_t leader_count(uint32_t id, bool in, uint32_t* shared) {
    const uint32_t lead = __builtin_amdgcn_readfirstlane(in ? id : 0xFFFFFFFFu);
    const uint64_t m = ballot(in && id == lead);
    *shared = popc64(m);
    if (!(m & (m - 1))) return in ? 1u : 0u;  // at most one lane holds the leader's bucket
    if (in && id == lead) return lanes_below(m) == 0 ? popc64(m) : 0u;
    return in ? 1u : 0u;
}

// Below this many lanes sharing the leader's bucket in a vector's first
// element, a wave counts the vector's other elements one lane at a time:
// spread keys then pay one leader check per vector, not one per key.
constexpr uint32_t kSkewLanes = 4;

// N compressed-histogram adds issued together: every returning LDS add is in
// flight before any carry is examined, so a lane waits for LDS once per N
// keys rather than once per key (a carry check between adds would order
// them).  c[e] == 0 adds nothing and cannot carry; such an add goes to a
// word picked by the lane (not the key's, which may be a hot one) so that it
// costs no same-address conflict.  Each add still sees its own old word, so
// every wrap is counted by exactly one add.  cnt holds 2^15 words.
template <int N>
__device__ __forceinline__ void hist16_add_n(uint32_t* cnt, const uint32_t* key, const uint32_t* c,
                                             uint32_t* wrap_lo, uint32_t* wrap_word) {
    uint32_t old[N], inc[N];
#pragma unroll
    for (int e = 0; e < N; ++e) {
        inc[e] = (key[e] & 1u) ? (c[e] << 16) : c[e];
        const uint32_t w = c[e] ? key[e] >> 1 : (threadIdx.x + 64u * e) & 0x7FFFu;
        old[e] = atomicAdd(&cnt[w], inc[e]);
    }
#pragma unroll
    for (int e = 0; e < N; ++e) {
        const bool word_wrap = (old[e] + inc[e]) < old[e];
        const bool lo_wrap = ((old[e] & 0xFFFFu) + (inc[e] & 0xFFFFu)) > 0xFFFFu;
        if (__builtin_expect(word_wrap, 0)) atomicAdd(&wrap_word[key[e] >> 1], 1u);
        if (__builtin_expect(lo_wrap, 0)) atomicAdd(&wrap_lo[key[e] >> 1], 1u);
    }
}

// N compressed-histogram adds of one count each (spread keys, every one in
// range).  An add of one can carry out of a 16-bit half only if that half
// read 0xFFFF, so one compare per add screens for wraps; the exact tests of
// hist16_add then run only in a wave where some lane saw a full half.  With
// a tile row `tc` (128 words of packed 16-bit counts of the low 8 bits) each
// key is counted there as well: its half there is the same as in `cnt`
// (bit 0 of the key).  Every add is issued before any result is examined.
template <int N>
__device__ __forceinline__ void hist16_add_ones(uint32_t* cnt, const uint32_t* key, uint32_t* tc,
                                                uint32_t* wrap_lo, uint32_t* wrap_word) {
    uint32_t old[N], sft[N];
#pragma unroll
    for (int e = 0; e < N; ++e) {
        sft[e] = (key[e] & 1u) << 4;
        old[e] = atomicAdd(&cnt[key[e] >> 1], 1u << sft[e]);
    }
    if (tc) {
#pragma unroll
        for (int e = 0; e < N; ++e) atomicAdd(&tc[(key[e] & 0xFFu) >> 1], 1u << sft[e]);
    }
    bool full = false;
#pragma unroll
    for (int e = 0; e < N; ++e) full |= ((old[e] >> sft[e]) & 0xFFFFu) == 0xFFFFu;
    if (__builtin_expect(full, 0)) {
#pragma unroll
        for (int e = 0; e < N; ++e) {
            const uint32_t inc = 1u << sft[e];
            const bool word_wrap = (old[e] + inc) < old[e];
            const bool lo_wrap = ((old[e] & 0xFFFFu) + (inc & 0xFFFFu)) > 0xFFFFu;
            if (word_wrap) atomicAdd(&wrap_word[key[e] >> 1], 1u);
            if (lo_wrap) atomicAdd(&wrap_lo[key[e] >> 1], 1u);
        }
    }
}

// Exclusive scan of one value per thread over the first 256 threads of a
// block (4 waves); every thread of the block must call it.  `wsum` is LDS
// scratch of at least 4 words.  Returns the exclusive prefix for threads
// < 256 and the total in *total (all threads).
template <typename T>
__device__ __forceinline__ T scan256_exclusive(T x, T* wsum, T* total) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    T inc = x;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        T y = __shfl_up(inc, off, 64);
        if (lane >= off) inc += y;
    }
    if (wave < 4 && lane == 63) wsum[wave] = inc;
    __syncthreads();
    T before = 0, all = 0;
#pragma unroll
    for (int w = 0; w < 4; ++w) {
        T s = wsum[w];
        if (w < wave) before += s;
        all += s;
    }
    *total = all;
    __syncthreads();
    return before + inc - x;
}

// Stable rank of one item per lane among the lanes of this wave: every
// valid lane ORs its lane bit into peers[d] (LDS, one 64-bit word per
// digit value, all zero on entry), so the word read back is the set of
// lanes sharing its digit whatever order the ORs took; the lowest of them
// clears the word and advances cnt[d], the wave's running count of d.
// Returns (count of d before this item) + (peers below this lane).
// FULL: every lane is valid (no lane masking at all).  The OR is waited for
// before the word is read back, and the leader's writes before the next
// item; without either wait the sort measured the same (the LDS runs a
// wave's operations in order, so the waits are for pacing, not ordering).
constexpr uint32_t kLgkmWait0 = 0xC07F;  // s_waitcnt lgkmcnt(0), other counters free
template <bool FULL = false>
__device__ __forceinline__ uint32_t wave_rank(uint32_t d, bool valid, uint64_t* peers_w,
                                              uint32_t* cnt_w) {
    if constexpr (FULL) {
        atomicOr(&peers_w[d], 1ull << (threadIdx.x & 63));
        __builtin_amdgcn_s_waitcnt(kLgkmWait0);
        __builtin_amdgcn_wave_barrier();
        const uint64_t peers = peers_w[d];
        const uint32_t before = cnt_w[d];
        __builtin_amdgcn_wave_barrier();
        const uint32_t below = lanes_below(peers);
        const uint32_t rank = before + below;
        if (below == 0) {
            peers_w[d] = 0;
            cnt_w[d] = before + popc64(peers);
        }
        __builtin_amdgcn_s_waitcnt(kLgkmWait0);
        __builtin_amdgcn_wave_barrier();
        return rank;
    } else {
        const uint64_t lane_bit = 1ull << (threadIdx.x & 63);
        if (valid) atomicOr(&peers_w[d], lane_bit);
        __builtin_amdgcn_wave_barrier();
        uint64_t peers = 0;
        uint32_t before = 0;
        if (valid) {
            peers = peers_w[d];
            before = cnt_w[d];
        }
        __builtin_amdgcn_wave_barrier();
        const uint32_t below = lanes_below(peers);
        if (valid && below == 0) {
            peers_w[d] = 0;
            cnt_w[d] = before + popc64(peers);
        }
        __builtin_amdgcn_wave_barrier();
        return before + below;
    }
}

// number of set bits of a lane mask, counted as two 32-bit halves so that
// comparisons on it stay scalar
__device__ __forceinline__ uint32_t popc_mask(uint64_t m) {
    return (uint32_t)__builtin_popcount((uint32_t)m) + (uint32_t)__builtin_popcount((uint32_t)(m >> 32));
}

// wave_rank with a fast path for the digit of the wave's first valid lane:
// when at least kRankLeaderLanes lanes hold it (presorted, reverse-sorted,
// hot-key or skewed input) they are ranked by their position among
// themselves, so they never touch the LDS word every one of them would OR
// into (a same-address conflict as wide as the group), and only the other
// lanes, if any, are ranked by wave_rank, which reads and updates other
// digits' counts only.  Valid lanes must be a prefix of the wave (lane 0
// then holds the first valid digit whenever any lane is valid).
constexpr uint32_t kRankLeaderLanes = 8;
template <bool FULL = false>
__device__ __forceinline__ uint32_t wave_rank_uniform_first(uint32_t d, bool valid, uint64_t* peers_w,
                                                            uint32_t* cnt_w) {
    const uint32_t d0 = __builtin_amdgcn_readfirstlane(d);
    const uint64_t m = ballot((FULL || valid) && d == d0);
    if (popc_mask(m) >= kRankLeaderLanes) {
        const uint64_t vm = FULL ? ~0ull : ballot(valid);
        const bool mine = (FULL || valid) && d == d0;
        const uint32_t before = cnt_w[d0];
        const uint32_t below = lanes_below(m);
        __builtin_amdgcn_wave_barrier();
        if (mine && below == 0) cnt_w[d0] = before + popc64(m);
        __builtin_amdgcn_wave_barrier();
        if (m == vm) return before + below;
        const uint32_t r = wave_rank<false>(d, (FULL || valid) && !mine, peers_w, cnt_w);
        return mine ? before + below : r;
    }
    return wave_rank<FULL>(d, valid, peers_w, cnt_w);
}

}  // namespace fs
