/*
 * oracle.c -- plain, slow, obviously correct CPU reference for the sort.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
 * baseline leg of the benchmark may load this library.  The product path
 * (the HIP library) never links, calls or includes anything from here, and
 * nothing here is shared with it.
 *
 * What it computes (paper: "FractalSortCPU", arXiv 2605.10390):
 *   - Radix sorting is split into a histogram phase, a prefix-sum phase and a
 *     stable scatter phase (Section II, Related Work).
 *   - A histogram node counts the keys in its subtree; the leaf of a key is
 *     reached by following the key's bits (Section III-B.1 "Fractal RMW",
 *     Algorithm 1).  For a d-bit digit the leaves are the 2^d digit values, so
 *     a leaf counter is the plain count of keys with that digit value.
 *   - The index of a value is the number of keys smaller than it, i.e. the
 *     exclusive prefix sum of the leaf counters (Algorithm 3, GetIndex).
 *   - The item at a sorted position is the smallest value whose inclusive
 *     prefix exceeds the position (Algorithm 2, GetItem).
 *   - When the histogram covers every key bit, the sorted array is the
 *     histogram written out bin by bin (Algorithm 5 with no trailing bits).
 *
 * Readings where the paper is silent: keys are unsigned and sorted
 * ascending; pairs are sorted stably (equal keys keep input order).  The
 * sort is a textbook least-significant-digit counting sort with 8-bit
 * digits and 64-bit counts: histogram, exclusive prefix, then a scatter that
 * walks the input in order, which is what makes it stable.
 *
 * oracle_sort_mt is the same sort split over threads, for timing the CPU
 * baseline only: each thread counts its contiguous chunk, the blocks are
 * laid out digit value by digit value and, within one, thread by thread,
 * and each thread then places its own chunk in order.  Chunks are in input
 * order, so equal keys still keep their input order (tested byte-equal to
 * oracle_sort).
 *
 * Build: gcc -O2 -shared -fPIC -pthread oracle.c -o liboracle.so (build.py).
 * Planted-mistake builds (tests only): -DORACLE_PLANT_<NAME>, see below.
 */
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_OK 0
#define ORACLE_BAD_ARG 1
#define ORACLE_NO_MEMORY 2

/* Read key i of an array of unsigned keys that are key_bytes wide. */
static uint64_t key_at(const void *keys, uint64_t i, int key_bytes)
{
    switch (key_bytes) {
#ifdef ORACLE_PLANT_KEY8_READS_16
    /* reads an 8-bit key array with a 16-bit stride */
    case 1: return ((const uint16_t *)keys)[i];
#else
    case 1: return ((const uint8_t *)keys)[i];
#endif
    case 2: return ((const uint16_t *)keys)[i];
    case 4: return ((const uint32_t *)keys)[i];
    default: return ((const uint64_t *)keys)[i];
    }
}

/* Copy element i of src to element j of dst, both elem_bytes wide. */
static void move_elem(void *dst, uint64_t j, const void *src, uint64_t i, int elem_bytes)
{
    memcpy((char *)dst + j * (uint64_t)elem_bytes,
           (const char *)src + i * (uint64_t)elem_bytes, (size_t)elem_bytes);
}

static int valid_key_bytes(int kb) { return kb == 1 || kb == 2 || kb == 4 || kb == 8; }

/*
 * Leaf counters of the digit that starts at bit `shift` and is `bits` wide
 * (Section III-B.1, Algorithm 1): hist[b] = #{ i : digit(key_i) == b } for
 * b in [0, 2^bits).  bits <= 16.
 */
int oracle_histogram(const void *keys, uint64_t n, int key_bytes, int shift, int bits,
                     uint64_t *hist)
{
    if (!valid_key_bytes(key_bytes) || bits < 1 || bits > 16 || shift < 0 ||
        shift + bits > 8 * key_bytes || (n && !keys) || !hist)
        return ORACLE_BAD_ARG;
    uint64_t nb = (uint64_t)1 << bits, mask = nb - 1;
    for (uint64_t b = 0; b < nb; ++b) hist[b] = 0;
    for (uint64_t i = 0; i < n; ++i) {
        uint64_t d = (key_at(keys, i, key_bytes) >> shift) & mask;
#ifdef ORACLE_PLANT_HIST_OFF_BY_ONE
        d = (d + 1) & mask;
#endif
        hist[d] += 1;
    }
    return ORACLE_OK;
}

/*
 * Exclusive prefix of the leaf counters (Algorithm 3, GetIndex):
 * prefix[b] = sum of hist[b'] for b' < b, and prefix[nb] = total.
 */
int oracle_exclusive_scan(const uint64_t *hist, uint64_t nb, uint64_t *prefix)
{
    if (!hist || !prefix) return ORACLE_BAD_ARG;
    uint64_t run = 0;
    for (uint64_t b = 0; b < nb; ++b) {
#ifdef ORACLE_PLANT_INCLUSIVE_SCAN
        run += hist[b];
        prefix[b] = run;
#else
        prefix[b] = run;
        run += hist[b];
#endif
    }
    prefix[nb] = run;
    return ORACLE_OK;
}

/*
 * Item at sorted position `index` (Algorithm 2, GetItem): the smallest value
 * v whose inclusive prefix sum(hist[0..v]) exceeds index.  Returns nb when
 * index >= total (the paper's defaultVal).
 */
uint64_t oracle_select(const uint64_t *hist, uint64_t nb, uint64_t index)
{
    uint64_t run = 0;
    for (uint64_t v = 0; v < nb; ++v) {
        run += hist[v];
        if (run > index) return v;
    }
    return nb;
}

/*
 * Sorted array from a histogram that covers every key bit (Algorithm 5 with
 * no trailing bits): out[i] = v for prefix[v] <= i < prefix[v+1].
 */
int oracle_expand(const uint64_t *hist, uint64_t nb, void *out, int key_bytes)
{
    if (!valid_key_bytes(key_bytes) || !hist) return ORACLE_BAD_ARG;
    uint64_t i = 0;
    for (uint64_t v = 0; v < nb; ++v) {
        for (uint64_t c = 0; c < hist[v]; ++c, ++i) {
            switch (key_bytes) {
            case 1: ((uint8_t *)out)[i] = (uint8_t)v; break;
            case 2: ((uint16_t *)out)[i] = (uint16_t)v; break;
            case 4: ((uint32_t *)out)[i] = (uint32_t)v; break;
            default: ((uint64_t *)out)[i] = v; break;
            }
        }
    }
    return ORACLE_OK;
}

/*
 * Stable ascending sort of unsigned keys, with an optional payload moved
 * alongside (vals_in/vals_out may be NULL when val_bytes == 0).
 *
 * Least-significant-digit first, 8-bit digits.  For each digit: count the
 * digit values (histogram), take the exclusive prefix (where each digit
 * value's block starts), then walk the input in order and place every
 * element at the next free slot of its block (stable scatter).
 */
int oracle_sort(const void *keys_in, void *keys_out, const void *vals_in, void *vals_out,
                uint64_t n, int key_bytes, int val_bytes)
{
    if (!valid_key_bytes(key_bytes)) return ORACLE_BAD_ARG;
    if (val_bytes != 0 && val_bytes != 4 && val_bytes != 8) return ORACLE_BAD_ARG;
    if (n && (!keys_in || !keys_out)) return ORACLE_BAD_ARG;
    if (n && val_bytes && (!vals_in || !vals_out)) return ORACLE_BAD_ARG;
    if (n == 0) return ORACLE_OK;

    /* Two buffers per array; pass p reads src and writes dst. */
    void *kbuf[2], *vbuf[2] = {NULL, NULL};
    kbuf[0] = malloc(n * (uint64_t)key_bytes);
    kbuf[1] = malloc(n * (uint64_t)key_bytes);
    if (val_bytes) {
        vbuf[0] = malloc(n * (uint64_t)val_bytes);
        vbuf[1] = malloc(n * (uint64_t)val_bytes);
    }
    if (!kbuf[0] || !kbuf[1] || (val_bytes && (!vbuf[0] || !vbuf[1]))) {
        free(kbuf[0]); free(kbuf[1]); free(vbuf[0]); free(vbuf[1]);
        return ORACLE_NO_MEMORY;
    }
    memcpy(kbuf[0], keys_in, n * (uint64_t)key_bytes);
    if (val_bytes) memcpy(vbuf[0], vals_in, n * (uint64_t)val_bytes);

    uint64_t hist[256], start[257];
    int cur = 0;
    int digits = key_bytes;
#ifdef ORACLE_PLANT_SKIP_TOP_DIGIT
    digits -= 1;
#endif
    for (int j = 0; j < digits; ++j) {
        const void *ks = kbuf[cur];
        void *kd = kbuf[1 - cur];
        oracle_histogram(ks, n, key_bytes, 8 * j, 8, hist);
        oracle_exclusive_scan(hist, 256, start);
#ifdef ORACLE_PLANT_UNSTABLE
        /* walks the input backwards but fills blocks from their starts, so
           equal keys come out in reverse input order */
        for (uint64_t ii = n; ii-- > 0;) {
            uint64_t d = (key_at(ks, ii, key_bytes) >> (8 * j)) & 0xFF;
            uint64_t slot = start[d]++;
            move_elem(kd, slot, ks, ii, key_bytes);
            if (val_bytes) move_elem(vbuf[1 - cur], slot, vbuf[cur], ii, val_bytes);
        }
#else
        for (uint64_t i = 0; i < n; ++i) {
            uint64_t d = (key_at(ks, i, key_bytes) >> (8 * j)) & 0xFF;
            uint64_t slot = start[d]++;
            move_elem(kd, slot, ks, i, key_bytes);
#ifdef ORACLE_PLANT_PAYLOAD_HALF
            /* moves only the low 4 bytes of an 8-byte payload */
            if (val_bytes) move_elem(vbuf[1 - cur], slot, vbuf[cur], i, val_bytes == 8 ? 4 : val_bytes);
#else
            if (val_bytes) move_elem(vbuf[1 - cur], slot, vbuf[cur], i, val_bytes);
#endif
        }
#endif
        cur = 1 - cur;
    }
    memcpy(keys_out, kbuf[cur], n * (uint64_t)key_bytes);
    if (val_bytes) memcpy(vals_out, vbuf[cur], n * (uint64_t)val_bytes);
    free(kbuf[0]); free(kbuf[1]); free(vbuf[0]); free(vbuf[1]);
    return ORACLE_OK;
}

#define ORACLE_MAX_THREADS 256

struct mt_job {
    const void *ks, *vs;
    void *kd, *vd;
    uint64_t lo, hi;
    int key_bytes, val_bytes, shift;
    uint64_t count[256]; /* this chunk's digit counts, then its next slots */
};

static void *mt_count(void *arg)
{
    struct mt_job *j = (struct mt_job *)arg;
    memset(j->count, 0, sizeof j->count);
    for (uint64_t i = j->lo; i < j->hi; ++i)
        j->count[(key_at(j->ks, i, j->key_bytes) >> j->shift) & 0xFF]++;
    return NULL;
}

static void *mt_place(void *arg)
{
    struct mt_job *j = (struct mt_job *)arg;
    for (uint64_t i = j->lo; i < j->hi; ++i) {
        uint64_t slot = j->count[(key_at(j->ks, i, j->key_bytes) >> j->shift) & 0xFF]++;
        move_elem(j->kd, slot, j->ks, i, j->key_bytes);
        if (j->val_bytes) move_elem(j->vd, slot, j->vs, i, j->val_bytes);
    }
    return NULL;
}

static int mt_run(void *(*fn)(void *), struct mt_job *jobs, int threads)
{
    pthread_t tid[ORACLE_MAX_THREADS];
    int started = 0, rc = ORACLE_OK;
    for (; started < threads; ++started)
        if (pthread_create(&tid[started], NULL, fn, &jobs[started]) != 0) break;
    for (int t = started; t < threads; ++t) fn(&jobs[t]); /* run here what could not start */
    for (int t = 0; t < started; ++t)
        if (pthread_join(tid[t], NULL) != 0) rc = ORACLE_BAD_ARG;
    return rc;
}

/* oracle_sort over `threads` threads (1..ORACLE_MAX_THREADS); same result. */
int oracle_sort_mt(const void *keys_in, void *keys_out, const void *vals_in, void *vals_out,
                   uint64_t n, int key_bytes, int val_bytes, int threads)
{
    if (!valid_key_bytes(key_bytes) || threads < 1 || threads > ORACLE_MAX_THREADS) return ORACLE_BAD_ARG;
    if (val_bytes != 0 && val_bytes != 4 && val_bytes != 8) return ORACLE_BAD_ARG;
    if (n && (!keys_in || !keys_out)) return ORACLE_BAD_ARG;
    if (n && val_bytes && (!vals_in || !vals_out)) return ORACLE_BAD_ARG;
    if (n == 0) return ORACLE_OK;
    if ((uint64_t)threads > n) threads = (int)n;

    void *kbuf[2], *vbuf[2] = {NULL, NULL};
    kbuf[0] = malloc(n * (uint64_t)key_bytes);
    kbuf[1] = malloc(n * (uint64_t)key_bytes);
    if (val_bytes) {
        vbuf[0] = malloc(n * (uint64_t)val_bytes);
        vbuf[1] = malloc(n * (uint64_t)val_bytes);
    }
    struct mt_job *jobs = calloc((size_t)threads, sizeof *jobs);
    if (!kbuf[0] || !kbuf[1] || (val_bytes && (!vbuf[0] || !vbuf[1])) || !jobs) {
        free(kbuf[0]); free(kbuf[1]); free(vbuf[0]); free(vbuf[1]); free(jobs);
        return ORACLE_NO_MEMORY;
    }
    memcpy(kbuf[0], keys_in, n * (uint64_t)key_bytes);
    if (val_bytes) memcpy(vbuf[0], vals_in, n * (uint64_t)val_bytes);

    int cur = 0, rc = ORACLE_OK;
    for (int j = 0; j < key_bytes && rc == ORACLE_OK; ++j) {
        for (int t = 0; t < threads; ++t) {
            jobs[t].ks = kbuf[cur];
            jobs[t].kd = kbuf[1 - cur];
            jobs[t].vs = vbuf[cur];
            jobs[t].vd = vbuf[1 - cur];
            jobs[t].lo = n * (uint64_t)t / (uint64_t)threads;
            jobs[t].hi = n * (uint64_t)(t + 1) / (uint64_t)threads;
            jobs[t].key_bytes = key_bytes;
            jobs[t].val_bytes = val_bytes;
            jobs[t].shift = 8 * j;
        }
        rc = mt_run(mt_count, jobs, threads);
        /* blocks: digit value major, thread minor (exclusive prefix) */
        uint64_t run = 0;
        for (int b = 0; b < 256; ++b)
            for (int t = 0; t < threads; ++t) {
                uint64_t c = jobs[t].count[b];
                jobs[t].count[b] = run;
                run += c;
            }
        if (rc == ORACLE_OK) rc = mt_run(mt_place, jobs, threads);
        cur = 1 - cur;
    }
    if (rc == ORACLE_OK) {
        memcpy(keys_out, kbuf[cur], n * (uint64_t)key_bytes);
        if (val_bytes) memcpy(vals_out, vbuf[cur], n * (uint64_t)val_bytes);
    }
    free(kbuf[0]); free(kbuf[1]); free(vbuf[0]); free(vbuf[1]); free(jobs);
    return rc;
}

/*
 * Independent segments (each sorted as if alone).  keys/vals are packed
 * back to back; seg_len[s] elements per segment; key_bytes per segment.
 * Segment s starts at byte offset seg_key_off[s] (and seg_val_off[s]).
 */
int oracle_sort_segments(const void *keys_in, void *keys_out, const void *vals_in, void *vals_out,
                         uint64_t num_segments, const uint64_t *seg_len, const int *seg_key_bytes,
                         const uint64_t *seg_key_off, const uint64_t *seg_val_off, int val_bytes)
{
    for (uint64_t s = 0; s < num_segments; ++s) {
        const char *ki = (const char *)keys_in + seg_key_off[s];
        char *ko = (char *)keys_out + seg_key_off[s];
        const char *vi = val_bytes ? (const char *)vals_in + seg_val_off[s] : NULL;
        char *vo = val_bytes ? (char *)vals_out + seg_val_off[s] : NULL;
        int rc = oracle_sort(ki, ko, vi, vo, seg_len[s], seg_key_bytes[s], val_bytes);
        if (rc) return rc;
    }
    return ORACLE_OK;
}
