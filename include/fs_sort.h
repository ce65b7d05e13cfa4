/*
 * fs_sort.h -- C ABI of the MI355X (gfx950) compressed-histogram radix sort.
 *
 * The operation is the one stated in "FractalSortCPU: Bandwidth-Efficient
 * Compressed Radix Sort on CPU" (arXiv 2605.10390): sort n keys of p bits.
 * Section II splits radix sorting into a histogram phase, a prefix-sum phase
 * and a stable scatter phase; Section III builds the histogram as a tree of
 * narrow counters (Fractal RMW, Algorithm 1; counter width tapering,
 * Section III-D.1), reads ranks from it as prefix sums (GetIndex,
 * Algorithm 3) and, when the histogram covers every key bit, writes the
 * sorted array straight from it (Algorithm 5).  Where the paper is silent
 * this library fixes: keys are unsigned integers, order is ascending, and
 * payloads follow their keys stably (equal keys keep their input order), so
 * every result is unique.
 *
 * Conventions shared by every call:
 *   - Pointers named d_* / keys_* / vals_* / workspace are DEVICE pointers
 *     (hipMalloc memory of the current device).  Arrays are dense and
 *     little-endian: element i of a key array sits at byte i * key_bits/8.
 *   - The caller owns every buffer, including the workspace.  The library
 *     never allocates or frees caller memory and keeps no pointer after a
 *     call returns.
 *   - `stream` is a hipStream_t (NULL = the default stream).  Calls only
 *     enqueue work on it and return without synchronising; results are
 *     ready when the stream reaches that point.  Calls on different streams
 *     with different workspaces may run concurrently.
 *   - Workspace query: pass workspace == NULL and the call writes the number
 *     of workspace bytes it needs to *workspace_bytes, launches nothing and
 *     returns FS_OK.  Otherwise *workspace_bytes is the size of the buffer
 *     passed; too small gives FS_ERR_WORKSPACE_TOO_SMALL.  The workspace
 *     must be 256-byte aligned.  Its contents on entry do not matter; on
 *     exit its first 32-bit word is 0 unless a device-side bounded wait gave
 *     up (a library defect), in which case the output is not valid.
 *   - Errors are status codes; nothing aborts.  A NULL pointer with n > 0,
 *     an unsupported width, overlapping input and output ranges, or an
 *     unaligned workspace give FS_ERR_INVALID_ARG and launch nothing.  A
 *     failed kernel launch gives FS_ERR_DEVICE.  n == 0 is FS_OK and a
 *     no-op.  n may be as large as 2^36.
 */
#ifndef FS_SORT_H
#define FS_SORT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    FS_OK = 0,
    FS_ERR_INVALID_ARG = 1,
    FS_ERR_UNSUPPORTED = 2,
    FS_ERR_WORKSPACE_TOO_SMALL = 3,
    FS_ERR_DEVICE = 4
} fs_status;

/*
 * Flags of fs_sort_keys / fs_sort_pairs.
 *
 * FS_FLAG_CLOBBER_INPUT: the caller allows the sort to overwrite keys_in
 *   (and vals_in): the input arrays then serve as the second buffer of the
 *   passes, so the workspace holds no temporary copy of the keys and
 *   payloads (its size, as queried with the same flags, shrinks by about
 *   n * (key_bits / 8 + val_bytes) bytes).  On return the input arrays hold
 *   unspecified bytes.  When the number of digits that are not trivial is
 *   even, the last pass lands in the input arrays and one extra copy moves
 *   it to the output.  The result itself does not depend on this flag.
 *
 * Key order (the paper sorts p-bit keys of any precision, Section I; these
 * fix how the bits are compared).  No order flag: unsigned integers,
 * ascending.
 *   FS_FLAG_SIGNED      two's-complement signed integers.
 *   FS_FLAG_FLOAT       IEEE 754 binary16 / binary32 / binary64 (for 16-bit
 *                       keys also bfloat16, ordered by the same rule) in the
 *                       standard's totalOrder: -NaN < -inf < negatives < -0
 *                       < +0 < positives < +inf < +NaN, NaNs ordered by
 *                       payload.  Bits are never changed, so NaN payloads
 *                       and the sign of zero survive.
 *   FS_FLAG_DESCENDING  largest key first.  Stability is kept: equal keys
 *                       (same bits) stay in input order.
 * SIGNED and FLOAT exclude each other, FLOAT needs 16 bits or more; any
 * other bit is FS_ERR_INVALID_ARG.
 * fs_sort_segmented applies the order flags to every segment of the call;
 * it and fs_sort_keys_wide / fs_sort_pairs_wide accept CLOBBER_INPUT and
 * leave their inputs and workspace sizes as they are.  The stream and
 * out-of-core calls take order flags only (CLOBBER_INPUT there is
 * FS_ERR_INVALID_ARG).
 */
enum {
    FS_FLAG_NONE = 0,
    FS_FLAG_CLOBBER_INPUT = 1,
    FS_FLAG_SIGNED = 2,
    FS_FLAG_FLOAT = 4,
    FS_FLAG_DESCENDING = 8
};

/*
 * Stable ascending sort of n unsigned keys (Section II phases; for 16-bit
 * keys the whole sort is the compressed 2^16-bin histogram written out in
 * order, Algorithm 5 with no trailing bits).
 *   keys_in   device, n keys of key_bits bits (8, 16, 32 or 64); not modified
 *             unless flags has FS_FLAG_CLOBBER_INPUT.
 *   keys_out  device, n keys; must not overlap keys_in.
 *   flags     FS_FLAG_CLOBBER_INPUT and the key order (FS_FLAG_SIGNED,
 *             FS_FLAG_FLOAT, FS_FLAG_DESCENDING).  The workspace size
 *             depends on n, key_bits and CLOBBER_INPUT.
 */
fs_status fs_sort_keys(const void *keys_in, void *keys_out, uint64_t n, int key_bits,
                       unsigned flags, void *workspace, size_t *workspace_bytes, void *stream);

/*
 * fs_sort_keys for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same sort, bit for bit, with the workspace taken from a static device
 * array of FS_NOALLOC_SCRATCH_BYTES (64 MiB) inside the library instead of
 * from the caller.  Each GPU the library runs on holds its own copy of that
 * array from the first call on it until the process ends; the call makes
 * no hipMalloc, hipFree or other allocation.
 *   keys_in, keys_out, n, key_bits, flags  as for fs_sort_keys (the call
 *             stays asynchronous on `stream`, whose device must be current).
 *   err_out   NULL, or a device word that receives the call's error word
 *             (stream-ordered, after the sort; 0 = ok, otherwise the bits
 *             fs_sort_keys leaves in word 0 of its workspace).
 * Returns FS_ERR_WORKSPACE_TOO_SMALL, launching nothing, when the workspace
 * fs_sort_keys would query for (n, key_bits, flags) exceeds
 * FS_NOALLOC_SCRATCH_BYTES: 16-bit keys take about 34 MiB at any n; 32- and
 * 64-bit keys with FS_FLAG_CLOBBER_INPUT fit up to about 2^28 keys, without
 * it up to about 2^23 (32-bit) or 2^22 (64-bit) keys.  Other errors as for
 * fs_sort_keys.
 * Every call on one GPU uses that GPU's one array and leaves its contents
 * there; each call clears what must start at zero.  Calls that overlap in
 * time on one GPU (on different streams, or from different threads without
 * stream ordering between them) race on the array and give undefined
 * results: serialise them, or use fs_sort_keys with workspaces of their own.
 */
#define FS_NOALLOC_SCRATCH_BYTES (64ull << 20)
fs_status fs_sort_keys_noalloc(const void *keys_in, void *keys_out, uint64_t n, int key_bits,
                               unsigned flags, uint32_t *err_out, void *stream);

/*
 * Stable ascending sort of n (key, value) pairs: keys_out is keys_in in
 * ascending order and vals_out[i] is the value that came with keys_out[i];
 * equal keys keep their input order.  With vals_in[i] = i, vals_out is the
 * paper's index array (sorted position -> arrival position, Section III-G.3).
 *   keys_in/keys_out  device, n keys of key_bits bits (8, 16, 32, 64).
 *   vals_in/vals_out  device, n values of val_bytes bytes (4 or 8).
 * None of the four ranges may overlap another.  flags: FS_FLAG_CLOBBER_INPUT
 * (keys_in and vals_in may then be overwritten) and the key order, as for
 * fs_sort_keys.  For 16-bit keys the passes never store whole keys: the
 * first keeps only each key's high byte (one byte per key, in the
 * workspace) for the second, and the sorted keys are written from the
 * 2^16-bin histogram, so the workspace holds no key copy even without
 * CLOBBER_INPUT.
 */
fs_status fs_sort_pairs(const void *keys_in, void *keys_out, const void *vals_in, void *vals_out,
                        uint64_t n, int key_bits, int val_bytes, unsigned flags,
                        void *workspace, size_t *workspace_bytes, void *stream);

/*
 * Keys wider than 64 bits (the paper sorts keys of any precision p,
 * Section I; its radix passes run over the key from the least significant
 * digit up, Section II).  A key is key_words 64-bit words, word 0 the least
 * significant, so key i occupies words [i * key_words, (i + 1) * key_words)
 * of keys_in (little-endian throughout: a key is one little-endian integer
 * of 64 * key_words bits).  key_words is 1..64; 1 is the 64-bit sort.
 * The sort runs one round per word, least significant first: each round
 * stably sorts that word (order-mapped) paired with the permutation so far,
 * and the last permutation moves whole keys and payloads.  Results are
 * those of fs_sort_keys / fs_sort_pairs for a key of that width: stable,
 * in the order `flags` gives (FS_FLAG_SIGNED: two's complement over the
 * whole width; FS_FLAG_FLOAT: sign-magnitude over the whole width, e.g.
 * IEEE binary128 for two words; FS_FLAG_DESCENDING).
 *   keys_in / keys_out  device, n * key_words uint64 words, 8-byte aligned,
 *                       not overlapping.
 *   vals_in / vals_out  device, n values of val_bytes bytes (4 or 8).
 * The workspace holds two permutations, two word arrays and the workspace
 * of a 64-bit pair sort of n elements.
 */
fs_status fs_sort_keys_wide(const void *keys_in, void *keys_out, uint64_t n, int key_words, unsigned flags,
                            void *workspace, size_t *workspace_bytes, void *stream);
fs_status fs_sort_pairs_wide(const void *keys_in, void *keys_out, const void *vals_in, void *vals_out,
                             uint64_t n, int key_words, int val_bytes, unsigned flags, void *workspace,
                             size_t *workspace_bytes, void *stream);

/*
 * Leaf counters of every digit of the keys (the histogram of Section III-B,
 * Algorithm 1, merged across workgroups as in Section III-A.1/III-B):
 *   hist_out[j * 2^digit_bits + b] = #{ i : bits [j*digit_bits,
 *                                        (j+1)*digit_bits) of key i == b }
 * for j in [0, key_bits / digit_bits).  digit_bits is 8 or 16 (16 only for
 * 16-bit keys, which uses the compressed 2^16-bin histogram).  hist_out is a
 * device array of uint64 written in full.
 */
fs_status fs_digit_histograms(const void *keys, uint64_t n, int key_bits, int digit_bits,
                              uint64_t *hist_out, void *workspace, size_t *workspace_bytes,
                              void *stream);

/*
 * One segment of a batched segmented sort.  keys_in/keys_out (and
 * vals_in/vals_out when vals_in is not NULL) are device pointers to n
 * elements; key_bits is 16, 32 or 64; val_bytes is 0 (keys only), 4 or 8.
 */
typedef struct {
    const void *keys_in;
    void *keys_out;
    const void *vals_in;
    void *vals_out;
    uint64_t n;
    uint32_t key_bits;
    uint32_t val_bytes;
} fs_segment;

/*
 * Many independent sorts in one call (each segment's result is exactly what
 * fs_sort_keys / fs_sort_pairs gives for it alone).  Batching follows the
 * paper's batch processing (Sections III-C, IV-D): segments are binned by
 * length on the device and drained by persistent workgroups.
 *   d_segments        DEVICE array of num_segments descriptors, read on the
 *                     device (it may be written by earlier stream work).
 *   total_keys        sum of the segments' n (host-known, for sizing).
 *   max_segment_keys  the largest n (host-known, for sizing).
 * Segments may mix key widths and payload widths.  A segment's buffers must
 * not overlap each other or another segment's.  flags: the key order of
 * every segment (FS_FLAG_SIGNED / FS_FLAG_FLOAT / FS_FLAG_DESCENDING, as for
 * fs_sort_keys; each segment's sign bit is that of its own width).
 */
fs_status fs_sort_segmented(const fs_segment *d_segments, uint32_t num_segments,
                            uint64_t total_keys, uint64_t max_segment_keys, unsigned flags,
                            void *workspace, size_t *workspace_bytes, void *stream);

/*
 * Launch tuning of fs_sort_segmented.  Segments are binned by length and
 * width on the device (the paper sizes its batches empirically,
 * Section III-C); these fields choose, per bin, the digit width, the tile
 * size and how many workgroups work on one segment:
 *   small_max_keys[w]  w = 0, 1, 2 for 16-, 32-, 64-bit keys: segments of at
 *                      most this many keys are sorted by ONE workgroup with
 *                      8-bit digits entirely in LDS.  Clamped to what fits
 *                      in LDS for the segment's key and payload width;
 *                      values below 1024 are raised to 1024.
 *   expand16_min_keys  16-bit keys-only segments of at least this many keys
 *                      use ONE 16-bit digit instead: one workgroup builds the
 *                      segment's compressed 2^16-bin histogram in LDS and
 *                      writes the sorted keys from it (Sections III-A, III-E).
 *                      This bin is checked first.  0xFFFFFFFF disables it.
 *   expand16_split_keys  segments of that bin with at least this many keys
 *                      are split over several workgroups (parts of 2^18
 *                      keys whose histograms are merged in global memory);
 *                      values below 2^18 are raised to 2^18, 0xFFFFFFFF
 *                      never splits.
 *   expand16_wgs_per_cu  workgroups per compute unit of that bin, 1..2.
 *   large_wg_max_keys  remaining segments of at most this many keys are
 *                      sorted by ONE workgroup each, with 8-bit digits and
 *                      passes through global memory (tiles of 256 *
 *                      tile_items keys walked in order; no look-back).  0
 *                      disables it.
 *   tile_items, tile_threads  the remaining (large) segments are sorted
 *                      with 8-bit digits by many workgroups, in tiles of
 *                      tile_threads * tile_items keys; tile_items is 8 or
 *                      16, tile_threads (the workgroup size) 256 or 512.
 *   large_wgs_per_cu   workgroups per compute unit of the large-segment
 *                      histogram and scatter launches, 1..8.
 *   small_wgs_per_cu   workgroups per compute unit of the LDS bin, 1..4.
 * Every setting gives bit-identical results; only the speed differs.
 */
typedef struct {
    uint32_t small_max_keys[3];
    uint32_t expand16_min_keys;
    uint32_t expand16_split_keys;
    uint32_t expand16_wgs_per_cu;
    uint32_t large_wg_max_keys;
    uint32_t tile_items;
    uint32_t tile_threads;
    uint32_t large_wgs_per_cu;
    uint32_t small_wgs_per_cu;
} fs_seg_tuning;

/* Writes the built-in default tuning to *out.  NULL out: FS_ERR_INVALID_ARG. */
fs_status fs_segmented_default_tuning(fs_seg_tuning *out);

/*
 * Sets the process-wide tuning that fs_sort_segmented uses (copied; NULL
 * restores the defaults).  A field out of range gives FS_ERR_INVALID_ARG
 * and leaves the table unchanged.  Thread-safe; a call in flight keeps the
 * tuning it started with.
 */
fs_status fs_set_segmented_tuning(const fs_seg_tuning *tuning);

/* Reads the process-wide tuning into *out. */
fs_status fs_get_segmented_tuning(fs_seg_tuning *out);

/*
 * fs_sort_segmented with an explicit tuning (NULL = the process-wide one);
 * this is what an autotuner times.  Same arguments, results, workspace size
 * and errors as fs_sort_segmented; a field out of range gives
 * FS_ERR_INVALID_ARG.
 */
fs_status fs_sort_segmented_tuned(const fs_segment *d_segments, uint32_t num_segments,
                                  uint64_t total_keys, uint64_t max_segment_keys, unsigned flags,
                                  const fs_seg_tuning *tuning, void *workspace,
                                  size_t *workspace_bytes, void *stream);

/* Human-readable name of a status code (static storage). */
/*
 * Batch stream sorting of 16-bit keys (Section I, contribution 2; batches,
 * Section III-C; reconstruction from the counters, Algorithm 5 with no
 * trailing bits).  For 16-bit keys the 2^16-bin histogram is the whole
 * multiset, so batches that arrive one after another are sorted by adding
 * each one's histogram into a resident histogram and writing the sorted
 * keys from it once the stream ends; no batch has to stay resident.
 *
 * fs_hist16_accumulate: d_hist[v] += #{ i < n : keys[i] == v } for all
 *   v < 2^16.  keys: device, n 16-bit keys.  d_hist: device, 65536 uint64,
 *   8-byte aligned, caller-initialised (zero it before the first batch);
 *   must not overlap keys or the workspace.  Workspace as for every call
 *   (its size depends on n only).  n == 0 adds nothing.  flags: a key order
 *   (FS_FLAG_SIGNED / FS_FLAG_FLOAT / FS_FLAG_DESCENDING): the histogram
 *   then counts the order-mapped keys, bin v holding the keys of rank v in
 *   that order; every batch of one histogram, and its expansion, must use
 *   the same flags.
 */
fs_status fs_hist16_accumulate(const void *keys, uint64_t n, unsigned flags, uint64_t *d_hist, void *workspace,
                               size_t *workspace_bytes, void *stream);

/*
 * fs_hist16_prefix: exclusive prefix of a 2^16-bin histogram (GetIndex of
 *   every value, Algorithm 3): d_prefix[v] = sum of d_hist[u] for u < v,
 *   v = 0..65536, so d_prefix[65536] is the number of keys.  Both device,
 *   8-byte aligned, not overlapping (65536 and 65537 uint64).
 */
fs_status fs_hist16_prefix(const uint64_t *d_hist, uint64_t *d_prefix, void *stream);

/*
 * fs_expand16: positions [first, first + count) of the sorted multiset that
 *   d_prefix (from fs_hist16_prefix) describes: keys_out[i - first] = v for
 *   d_prefix[v] <= i < d_prefix[v + 1].  keys_out: device, count 16-bit
 *   keys, not overlapping d_prefix.  Positions at or beyond the total
 *   d_prefix[65536] are left unwritten.  Any range may be asked for, in any
 *   order, so the output can be produced in pieces.  flags: the key order
 *   the histogram was accumulated with (the keys written are the caller's
 *   bits).
 */
fs_status fs_expand16(const uint64_t *d_prefix, uint64_t first, uint64_t count, unsigned flags,
                      void *keys_out, void *stream);

/*
 * fs_sort16_host: ascending sort of n 16-bit keys that live in HOST memory
 *   (the input need not fit in device memory).  The keys are copied in
 *   batch_keys at a time through two device staging slots in the workspace
 *   and counted with fs_hist16_accumulate as they arrive; the sorted keys
 *   are then written back to h_keys_out through the same slots.
 *   h_keys_in / h_keys_out: host, n 16-bit keys; they may be the same
 *   buffer (in-place) but must not otherwise overlap.  Pinned host memory
 *   (hipHostMalloc) lets copies and counting overlap; pageable memory works
 *   at the copy speed of the runtime's staging.
 *   copy_stream / compute_stream: hipStream_t's for the copies and the
 *   kernels (they may be the same stream; NULL = the default stream).
 *   The workspace size depends on batch_keys only.  Unlike the other calls
 *   this one BLOCKS until h_keys_out holds the result (both streams are
 *   synchronised).  n == 0 is FS_OK and a no-op.  flags: key order, as for
 *   fs_sort_keys.
 */
fs_status fs_sort16_host(const void *h_keys_in, void *h_keys_out, uint64_t n, uint64_t batch_keys,
                         unsigned flags, void *workspace, size_t *workspace_bytes, void *copy_stream,
                         void *compute_stream);

/*
 * fs_sort_host: ascending sort of n 32- or 64-bit keys (key_bits) that live
 *   in HOST memory and need not fit in device memory (batch stream sorting,
 *   Section I contribution 2, for keys whose histogram is not the whole
 *   multiset).  An MSD spill over the host input, streamed through two
 *   staging slots of batch_keys keys:
 *     1. one read finds the bits on which keys differ;
 *     2. one read builds the compressed 2^16-bin histogram (Section III-B)
 *        of the 16 bits just below the highest such bit;
 *     3. consecutive bins are grouped into ranges of at most device_keys
 *        keys, in key order; for each range one more read gathers its keys
 *        on the device, fs_sort_keys sorts them, and they are copied to
 *        their place in h_keys_out.  A bin holding more than device_keys
 *        keys is split the same way by its next 16 bits (one more read for
 *        its histogram, restricted to its keys), down to the lowest bits,
 *        where such a bin is a single key value and is written out as a run
 *        of it.
 *   The input is read (number of ranges + number of histograms + 1) times.
 *   h_keys_in/h_keys_out: host, n keys, not overlapping (the input is read
 *   until the last range); pinned memory (hipHostMalloc) makes the copies
 *   asynchronous.  When every key is equal the input is copied.  The
 *   workspace size
 *   depends on batch_keys and device_keys.  Blocks until h_keys_out holds
 *   the result.  n == 0 is FS_OK and a no-op.  flags: key order, as for
 *   fs_sort_keys (the spill then works on order-mapped keys).
 */
fs_status fs_sort_host(const void *h_keys_in, void *h_keys_out, uint64_t n, int key_bits, uint64_t batch_keys,
                       uint64_t device_keys, unsigned flags, void *workspace, size_t *workspace_bytes,
                       void *copy_stream, void *compute_stream);

const char *fs_status_string(fs_status s);

#ifdef __cplusplus
}
#endif

#endif /* FS_SORT_H */
