/*
 * fs_profile.h -- per-kernel timing of the sort library (instrumentation).
 *
 * The paper reports sort latency as an average over repeated runs (Section
 * IV) and rates a sort by how much of the memory traffic it causes is
 * useful (bandwidth efficiency, Equation beff, Section IV-F.1).  To measure
 * that per kernel, the library can record a HIP event pair around every
 * kernel it launches, on the stream the kernel is launched on.
 *
 * Thread safety: the recorder is process-global and guarded by a mutex;
 * enabling it while calls are in flight on other threads is allowed (their
 * launches may or may not be recorded).
 */
#ifndef FS_PROFILE_H
#define FS_PROFILE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    FS_KERNEL_HISTOGRAM = 0, /* per-workgroup digit histograms (one read of the keys) */
    FS_KERNEL_PLAN = 1,      /* merge of histograms, prefix scans, pass plan */
    FS_KERNEL_SCATTER = 2,   /* one stable scatter pass over all keys */
    FS_KERNEL_EXPAND = 3,    /* 16-bit keys-only output written from the histogram */
    FS_KERNEL_AUX = 4,       /* clears and the copy of an all-trivial sort */
    FS_KERNEL_SEGMENTED = 5, /* batched segmented-sort kernels */
    FS_KERNEL_KINDS = 6
} fs_kernel_kind;

/* Start (on != 0) or stop recording; starting clears earlier records.
   Returns the previous state. */
int fs_profile_enable(int on);

/* Totals over the recorded launches of one kind: number of launches, keys
   they processed (the per-launch work unit), and summed event-measured
   duration in milliseconds.  Waits for the recorded events to complete.
   Returns 0, or -1 for an invalid kind or a failed event query. */
int fs_profile_read(int kind, uint64_t *launches, uint64_t *keys, double *total_ms);

#ifdef __cplusplus
}
#endif

#endif /* FS_PROFILE_H */
