// Host-side internals: workspace layout and kernel launchers.
#pragma once
#include <hip/hip_runtime.h>

#include "fs_sort.h"
#include "fs_device.hpp"
#include <stddef.h>
#include <stdint.h>

namespace fs {

// Histogram launch shapes.
constexpr int kHist16Threads = 1024;
constexpr int kHist16Unroll = 4;  // vectors per thread in flight in k_hist16c
constexpr int kHist16Words = 32768;  // 2^16 bins as packed 16-bit counter pairs
constexpr int kHist8Threads = 512;

struct ScatterShape {
    int threads;
    int items;
    int tile() const { return threads * items; }
};

// Offsets (bytes) of every region of a sort's workspace.
struct SortLayout {
    int key_bytes = 0, val_bytes = 0, digits = 0;
    bool expand16 = false;  // 16-bit keys only: compressed histogram + expansion
    bool pairs16 = false;   // 16-bit keys + payload: tiled passes, keys expanded at the end
    bool clobber = false;   // the input arrays are the passes' second buffer
    bool trie = false;      // 32/64-bit keys: the plan may take the sparse-trie window
    uint32_t hist_groups = 0;  // workgroups of the histogram kernel
    uint32_t hist16_groups = 0;
    uint32_t tile = 0, scatter_groups = 0;
    uint64_t tiles = 0, tile_blocks = 0, tile_supers = 0;
    size_t err = 0, plan = 0, hist = 0, base = 0, part = 0, wrap = 0, h16 = 0, p16 = 0, th = 0, bsum = 0,
           ssum = 0, sbase = 0, tile_tickets = 0, sink = 0, part16 = 0, tmp_keys = 0, tmp_vals = 0, total = 0,
           trie_list = 0, trie_count = 0, narrow = 0;
};

// clobber: the input arrays are the passes' second buffer (no temporary copy)
SortLayout sort_layout(uint64_t n, int key_bytes, int val_bytes, int num_cus, bool clobber = false);
int device_cu_count();

// ---- launchers (each returns hipGetLastError after enqueueing) ----------
hipError_t launch_fill_u32(uint32_t* p, uint64_t words, uint32_t value, hipStream_t s);
// zero up to four word ranges in one launch (ranges with words == 0 are skipped)
struct ZeroRanges {
    uint32_t* p[4] = {nullptr, nullptr, nullptr, nullptr};
    uint64_t words[4] = {0, 0, 0, 0};
};
hipError_t launch_zero(const ZeroRanges& r, hipStream_t s);

// pos, neg: key order masks (order_map); 0, 0 counts the keys as they are
hipError_t launch_hist16c(const uint16_t* keys, uint64_t n, uint32_t groups, uint32_t* part,
                          uint32_t* wrap_lo, uint32_t* wrap_word, hipStream_t s, uint32_t pos = 0,
                          uint32_t neg = 0);
hipError_t launch_merge16(const uint32_t* part, uint32_t groups, const uint32_t* wrap_lo,
                          const uint32_t* wrap_word, uint64_t* h16, hipStream_t s,
                          bool accumulate = false);
hipError_t launch_scan16(const uint64_t* h16, uint64_t* p16, hipStream_t s);
hipError_t launch_plan_from16(const uint64_t* h16, uint64_t n, uint64_t* hist, uint64_t* base,
                              uint32_t* plan, hipStream_t s, bool clobber = false);
hipError_t launch_hist8(const void* keys, uint64_t n, int key_bytes, uint32_t groups,
                        uint32_t* part, hipStream_t s);
hipError_t launch_plan8(const uint32_t* part, uint32_t groups, int digits, uint64_t n,
                        uint64_t* hist, uint64_t* base, uint32_t* plan, hipStream_t s);
hipError_t launch_reduce8(const uint32_t* part, uint32_t groups, int digits, uint64_t* hist,
                          hipStream_t s);
// writes sorted positions [first, first + count) (clipped to the total p16[65536]) to out,
// each value unmapped with the key order masks pos, neg (order_unmap)
hipError_t launch_expand16(const uint64_t* p16, uint16_t* out, uint64_t first, uint64_t count,
                           hipStream_t s, uint32_t pos = 0, uint32_t neg = 0);
// copies bytes from src to dst when plan[word] is set (kPlanCopy: the
// input is the result; kPlanCopyTmp: the temporary buffer is)
hipError_t launch_copy_if(const uint32_t* plan, const void* src, void* dst, uint64_t bytes,
                          hipStream_t s, int word = kPlanCopy);

// ---- tiled reduce-then-scan path (tiled.hip) -------------------------------
constexpr uint64_t kSuperBlock = 256;  // blocks per super-block of the offset scan
constexpr uint32_t kXcds = 8;          // tile groups of a scatter launch (one per XCD)
constexpr uint32_t kTicketStride = 32; // words between ticket counters (one 128-byte line each)
constexpr uint64_t kTrieMinKeys = 1ull << 22;  // sorts offered the sparse-trie plan
constexpr uint32_t kTrieLongMax = 1u << 20;    // capacity of the list of long trie runs

struct TiledArgs {
    const void* in_k;
    void* out_k;
    void* tmp_k;
    const void* in_v;
    void* out_v;
    void* tmp_v;
    uint64_t n;
    uint64_t tiles;         // ceil(n / tile)
    uint32_t tile;          // keys per tile (the scatter's threads * items)
    uint32_t block_tiles;   // tiles per block: 65536 / tile
    const uint32_t* plan;
    const uint64_t* base;   // plan: start of every digit value in each pass output
    uint32_t* th;           // [tiles][256] 16-bit counts of the pass digit, then block prefixes
    uint32_t* bsum;         // [blocks][256] block totals, then super-block prefixes
    uint32_t* ssum;         // [super-blocks][256] super-block totals
    uint64_t* sbase;        // [super-blocks][256] super-block starts in the pass output
    uint32_t* part;         // [groups][digits][256] first-pass workgroup totals
    uint32_t* tickets;      // [passes][kXcds][kTicketStride] tile tickets, zero on entry
    void* sink;             // 16 bytes that absorb the stores of out-of-range lanes
    uint32_t* err;
    uint64_t ord_pos = 0;   // key order masks (order_map); both 0: unsigned ascending
    uint64_t ord_neg = 0;
    uint64_t* trie_list = nullptr;   // sparse-trie plan: starts of runs longer than one thread sorts
    uint32_t* trie_count = nullptr;  // entries appended to trie_list (zero on entry)
    // 16-bit pair sorts: n bytes holding, in the order of the first pass's
    // output, the high byte of every (mapped) key.  The first pass writes
    // them instead of the keys; the second pass counts and scatters them as
    // one-byte keys (its digit), as the sorted keys themselves are rebuilt
    // from the 2^16-bin histogram.  Null for every other sort.
    uint8_t* narrow = nullptr;
};

ScatterShape tiled_shape(int key_bytes, int val_bytes);
int tiled_scatter_per_cu(int key_bytes, int val_bytes);
// tile counts of slot `pass`'s digit; `first`: the first read of the input,
// which also totals every digit per workgroup for the plan (slot 0 only)
hipError_t launch_tile_hist(const TiledArgs& a, int key_bytes, int pass, uint32_t groups, hipStream_t s,
                            bool first);
hipError_t launch_tile_offsets(const TiledArgs& a, int pass, hipStream_t s);
hipError_t launch_tile_plan(const uint32_t* part, uint32_t groups, int digits, uint64_t n, uint64_t* hist,
                            uint64_t* base, uint32_t* plan, hipStream_t s, bool clobber = false,
                            int trie_bits = 0);
// Sparse-trie fixup: sorts every run of keys that share their bits from
// plan[kPlanTrieShift] up by the trailing bits below (stable, payloads
// alongside), in place in buffer plan[kPlanFixBuf]; runs longer than one
// thread sorts are listed for launch_trie_longruns.
hipError_t launch_trie_fixup(const TiledArgs& a, int key_bytes, int val_bytes, hipStream_t s);
// Runs the fixup listed as too long for one thread: each is sorted in LDS by
// one workgroup when it holds at most kTrieLdsRun keys and is out of order;
// a longer run out of order switches on the fallback slots.
hipError_t launch_trie_longruns(const TiledArgs& a, int key_bytes, int val_bytes, hipStream_t s);
// 16-bit keys (pair sorts only) write just their high bytes to a.narrow
hipError_t launch_tile_scatter(const TiledArgs& a, int key_bytes, int val_bytes, int pass, uint32_t groups,
                               hipStream_t s);
// second pass of a 16-bit pair sort: the bytes in a.narrow are the keys
// (digit 0), only payloads are written; tiles as for 16-bit keys
hipError_t launch_tile_scatter_narrow(const TiledArgs& a, int val_bytes, int pass, uint32_t groups,
                                      hipStream_t s);
// a.narrow[i] = high byte of the mapped key i of the input, when the plan
// skips the first pass of a 16-bit pair sort and runs the second
hipError_t launch_narrow_copy(const TiledArgs& a, hipStream_t s);
hipError_t launch_tile_hist16(const TiledArgs& a, uint32_t groups, uint32_t* part16, uint32_t* wrap_lo,
                              uint32_t* wrap_word, hipStream_t s);

// order_map masks (pos, neg) of the key order flags for key_bits-wide keys;
// false for an unknown flag, SIGNED with FLOAT, or FLOAT with 8-bit keys
bool order_masks(unsigned flags, int key_bits, uint64_t* pos, uint64_t* neg);

// ---- multi-word keys (wide.hip) ---------------------------------------------
// perm_bytes: 4 or 8 (width of a permutation entry)
hipError_t launch_iota(void* perm, int perm_bytes, uint64_t n, hipStream_t s);
// out[i] = word w of key perm[i] (key i when perm is null) ^ (pos, or neg when the
// key's top word has its top bit set)
hipError_t launch_gather_word(const void* keys, uint32_t words, uint32_t w, const void* perm, int perm_bytes,
                              uint64_t* out, uint64_t n, uint64_t pos, uint64_t neg, hipStream_t s);
hipError_t launch_gather_keys(const void* keys_in, void* keys_out, uint32_t words, const void* perm, int perm_bytes,
                              uint64_t n, hipStream_t s);
hipError_t launch_gather_vals(const void* vals_in, void* vals_out, int val_bytes, const void* perm, int perm_bytes,
                              uint64_t n, hipStream_t s);

// ---- per-kernel event timing (include/fs_profile.h) ------------------------
void profile_mark(int kind, uint64_t keys, hipStream_t s, hipEvent_t* begin_out);
// While one exists on a thread, that thread's launches record no events.
struct ProfileSuspend {
    ProfileSuspend();
    ~ProfileSuspend();
    ProfileSuspend(const ProfileSuspend&) = delete;
    ProfileSuspend& operator=(const ProfileSuspend&) = delete;
};
void profile_close(int kind, uint64_t keys, hipStream_t s, hipEvent_t begin);

// Enqueue one launch, bracketed by timing events while profiling is on.
template <typename F>
hipError_t timed(int kind, uint64_t keys, hipStream_t s, F&& launch) {
    hipEvent_t b = nullptr;
    profile_mark(kind, keys, s, &b);
    const hipError_t r = launch();
    profile_close(kind, keys, s, b);
    return r;
}

// ---- batched segmented sort (segmented.hip) --------------------------------
constexpr uint32_t kSegSmallBytes = 32768;           // LDS bytes per buffer of a small segment
constexpr uint32_t kSegWaveMaxKeys = 64;  // segments this short take the wave bin
constexpr uint64_t kSegMaxKeys = (1ull << 23) - 1;  // largest segment (look-back counts are 23-bit)
constexpr uint32_t kSegMinSmallMax = 1024;         // least segment length a tuning may send to the large bin
constexpr uint32_t kSegMinTile = 2048;             // smallest large-segment tile (sizes the tile arrays)
constexpr uint32_t kX16Part = 1u << 18;            // keys per part of a long 16-bit-digit segment
constexpr uint32_t kX16MinSplit = 1u << 18;        // least segment length a tuning may split

// what a scatter pass needs of one tile of a large segment, in one 64-byte
// record so that a workgroup finds it with a single load
struct SegTileDesc {
    const void* kin;
    void* kout;
    const void* vin;
    void* vout;
    uint64_t n;      // segment length
    uint64_t eo;     // segment's offset in the temporary arrays
    uint32_t q;      // segment's position in its class list
    uint32_t t;      // tile index within the segment
    uint32_t plan[2];  // 8 bits per pass: active, source (bits 1-2), destination (bits 3-4)
};
static_assert(sizeof(SegTileDesc) == 64, "tile record is one 64-byte line");

struct SegCtx {
    const fs_segment* segs;
    uint32_t nseg;
    uint64_t max_seg;
    uint64_t total_keys;
    uint32_t max_tiles;
    uint32_t tile;          // keys per large-segment tile
    uint32_t small_max[3];  // per key width: longest segment of the LDS bin
    uint32_t expand_min;    // 16-bit keys-only segments this long take the 16-bit-digit bin
    uint32_t split_min;     //   and from this long get several workgroups
    uint32_t wg_max;        // large segments up to this long get one workgroup each
    uint32_t* err;
    uint32_t* ctr;          // queue counters, tile totals, tickets
    uint32_t* small_list;   // [nseg]
    uint32_t* wave_list;    // [nseg]: segments of at most kSegWaveMaxKeys keys
    uint32_t* expand_list;  // [nseg]: long segments from the front, the rest from the back
    uint32_t* x16_parts;    // [long segments + 1] part prefix
    uint32_t* x16_hist;     // [long segments][65536] exact bin counts
    uint32_t* large_list;   // [9][nseg]
    uint32_t* wg_list;      // [9][nseg]
    uint32_t* tile_prefix;  // [nseg + 1] (current class)
    uint64_t* elem_prefix;  // [nseg + 1] (current class)
    uint32_t* tile_seg;     // [max_tiles]
    uint32_t* hist;         // [large segments][8][256]
    uint32_t* plan;         // [large segments][9]
    uint32_t* state;        // [max_tiles][256]
    SegTileDesc* tdesc;     // [max_tiles]
    void* tmp_k;
    void* tmp_v;
    uint32_t ord = 0;                 // nonzero: keys compare through order_map
    uint64_t ord_pos[3] = {0, 0, 0};  // its masks per key width (16, 32, 64 bits)
    uint64_t ord_neg[3] = {0, 0, 0};
};
uint32_t seg_max_tiles(uint64_t total_keys, uint32_t nseg);
// checks a tuning's ranges (false: invalid)
bool seg_tuning_valid(const fs_seg_tuning& t);
hipError_t launch_segmented(const SegCtx& x, const fs_seg_tuning& t, hipStream_t s);

}  // namespace fs
