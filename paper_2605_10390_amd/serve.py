"""Continuous-batching sort server on one GPU.

The paper's batch stream sorting (Section I, contribution 2; Section IV-D)
sorts a stream of batches as they arrive.  Here requests are sort jobs of
mixed sizes and key widths arriving over time.  A host scheduler admits
jobs as execution slots (HIP streams, all at the default priority) and
device memory free up, under a fixed memory budget:

  * a job's device bytes are its input, its output and its workspace;
  * waiting jobs are admitted in arrival order; several waiting small jobs
    are merged into one fs_sort_segmented launch (continuous batching),
    a large job gets a slot of its own;
  * each slot's work ends with a HIP event; completions are found by
    polling the events, and free the job's memory and slot at once, so the
    next waiting jobs start while others are still running on the device;
  * a job that could never fit the budget is rejected instead of blocking
    the queue;
  * a job's input is already resident in device memory when it arrives
    (the caller attaches it as job.keys_in); the server allocates only its
    output and workspace;
  * the budget is real memory: one device buffer of budget_bytes is
    reserved when the server starts (Arena), and every launch's outputs and
    workspace are carved from it at admission and returned at completion,
    so the server never holds more than its budget whatever the caching
    allocator would keep;
  * after each launch the workspace's error word (word 0) is copied to a
    pinned host word of the slot; a job whose word is not 0 is marked
    failed (job.failed, job.error) and its output must not be used.

Every job's result is exactly what a stand-alone sort of it gives (the
segmented path sorts each segment independently and stably).

The admission logic (AdmissionPolicy) holds no device state and is tested
on the CPU; SortServer drives it with real device work.
"""
import collections
import time

import torch

from . import (SegmentBatch, Workspace, sort_keys, sort_keys_workspace_bytes,
               sort_segmented_workspace_bytes)

KEY_DTYPES = {16: torch.uint16, 32: torch.uint32, 64: torch.uint64}


class Job:
    """One sort request: n keys of key_bits bits drawn from `dist` with
    `seed`, arriving `arrival` seconds after the trace starts."""

    __slots__ = ("id", "key_bits", "n", "dist", "seed", "arrival", "admitted", "done", "batched",
                 "rejected", "failed", "error", "keys_in", "keys_out", "nbytes")

    def __init__(self, jid, key_bits, n, dist, seed, arrival):
        self.id, self.key_bits, self.n, self.dist, self.seed = jid, key_bits, int(n), dist, seed
        self.arrival = float(arrival)
        self.admitted = self.done = None
        self.batched = False
        self.rejected = False
        self.failed = False
        self.error = 0
        self.keys_in = self.keys_out = None
        self.nbytes = 0

    @property
    def latency(self):
        return None if self.done is None else self.done - self.arrival


class AdmissionPolicy:
    """Which waiting jobs start next (no device state; CPU-testable).

    cost(job) gives the job's device bytes.  pick(queue, free_bytes) returns
    the jobs to launch together on one free slot, in arrival order, or []
    when the head of the queue must wait for memory.
    """

    def __init__(self, budget_bytes, cost, small_keys=1 << 20, batch_jobs=64, batch_keys=1 << 24,
                 batch_overhead=lambda jobs: 0):
        self.budget = int(budget_bytes)
        self.cost = cost
        self.small_keys = small_keys
        self.batch_jobs = batch_jobs
        self.batch_keys = batch_keys
        self.batch_overhead = batch_overhead

    def fits_ever(self, job):
        return self.cost(job) <= self.budget

    def pick(self, queue, free_bytes):
        if not queue:
            return []
        head = queue[0]
        if head.n > self.small_keys:
            return [head] if self.cost(head) <= free_bytes else []
        # merge consecutive waiting small jobs (arrival order) into one launch
        group, total, keys = [], 0, 0
        for job in queue:
            if job.n > self.small_keys or len(group) >= self.batch_jobs:
                break
            if keys + job.n > self.batch_keys and group:
                break
            c = self.cost(job)
            if total + c + self.batch_overhead(group + [job]) > free_bytes:
                break
            group.append(job)
            total += c
            keys += job.n
        return group


class Arena:
    """First-fit allocator over one device buffer (the server's whole
    memory budget, reserved once).  Blocks are 256-byte aligned; freed
    blocks merge with free neighbours."""

    ALIGN = 256

    def __init__(self, nbytes, device):
        self.size = (int(nbytes) // self.ALIGN) * self.ALIGN
        self.buf = torch.empty(self.size, dtype=torch.uint8, device=device)
        self.free = [(0, self.size)]  # (offset, bytes), sorted by offset

    @classmethod
    def round(cls, nbytes):
        return max(cls.ALIGN, (int(nbytes) + cls.ALIGN - 1) // cls.ALIGN * cls.ALIGN)

    def alloc(self, nbytes):
        """Offset of a free block of nbytes (rounded up), or None."""
        nbytes = self.round(nbytes)
        for i, (o, sz) in enumerate(self.free):
            if sz >= nbytes:
                if sz == nbytes:
                    del self.free[i]
                else:
                    self.free[i] = (o + nbytes, sz - nbytes)
                return o
        return None

    def release(self, off, nbytes):
        nbytes = self.round(nbytes)
        i = 0
        while i < len(self.free) and self.free[i][0] < off:
            i += 1
        self.free.insert(i, (off, nbytes))
        if i + 1 < len(self.free) and off + nbytes == self.free[i + 1][0]:
            self.free[i] = (off, nbytes + self.free[i + 1][1])
            del self.free[i + 1]
        if i > 0 and self.free[i - 1][0] + self.free[i - 1][1] == off:
            self.free[i - 1] = (self.free[i - 1][0], self.free[i - 1][1] + self.free[i][1])
            del self.free[i]

    def view(self, off, nbytes, dtype):
        return self.buf[off:off + nbytes].view(dtype)


class SortServer:
    """Serves a trace of Jobs on one GPU with `slots` concurrent streams."""

    def __init__(self, device="cuda", budget_bytes=200 << 30, slots=4, small_keys=1 << 20,
                 batch_jobs=64, batch_keys=1 << 24, keep_outputs=False):
        self.device = torch.device(device)
        self.slots = [torch.cuda.Stream(self.device) for _ in range(slots)]  # default priority
        # one pinned host word per slot receives the error word of its launch
        self.err_host = torch.zeros(slots, dtype=torch.int32, pin_memory=True)
        self.arena = Arena(budget_bytes, self.device)
        self.keep_outputs = keep_outputs
        self.policy = AdmissionPolicy(budget_bytes, self._job_bytes, small_keys, batch_jobs,
                                      batch_keys, self._batch_overhead)
        self.used = 0
        self.peak_used = 0
        self.max_in_flight = 0
        self.launches = 0

    # -- memory accounting ---------------------------------------------------
    @staticmethod
    def _job_bytes(job):
        kb = job.key_bits // 8
        return 2 * job.n * kb + (sort_keys_workspace_bytes(job.n, job.key_bits)
                                 if job.n > 0 else 0)

    @staticmethod
    def _batch_overhead(jobs):
        if len(jobs) < 2:
            return 0
        return sort_segmented_workspace_bytes(len(jobs), sum(j.n for j in jobs),
                                              max(j.n for j in jobs))

    # -- device work --------------------------------------------------------
    def _launch(self, jobs, stream, slot, base):
        """Outputs and workspace are carved, in that order, from the arena
        block at `base` (its size is the group's budgeted bytes)."""
        off = base
        for j in jobs:
            if j.keys_in is None or j.keys_in.numel() != j.n or j.keys_in.dtype != KEY_DTYPES[j.key_bits]:
                raise ValueError(f"job {j.id}: keys_in must be a resident tensor of {j.n} "
                                 f"{j.key_bits}-bit keys")
            nb = j.n * (j.key_bits // 8)
            j.keys_out = self.arena.view(off, nb, KEY_DTYPES[j.key_bits])
            off += Arena.round(nb)
        ws = Workspace(self.device)
        with torch.cuda.stream(stream):
            if len(jobs) == 1 and not jobs[0].batched:
                ws.buf = self.arena.view(off, Arena.round(sort_keys_workspace_bytes(jobs[0].n, jobs[0].key_bits)),
                                         torch.uint8)
                sort_keys(jobs[0].keys_in, out=jobs[0].keys_out, workspace=ws)
            else:
                for j in jobs:
                    j.batched = True
                batch = SegmentBatch([(j.keys_in, j.keys_out, None, None) for j in jobs], device=self.device)
                ws.buf = self.arena.view(off, Arena.round(batch.workspace_bytes()), torch.uint8)
                batch.run(ws, stream=stream)
            self.err_host[slot:slot + 1].copy_(ws.buf[:4].view(torch.int32), non_blocking=True)
            ev = torch.cuda.Event()
            ev.record(stream)
        self.launches += 1
        return ev, ws

    # -- scheduling loop ----------------------------------------------------
    def serve(self, jobs, on_done=None, poll_sleep=0.0):
        """Run the trace (jobs sorted by arrival).  Returns the jobs with
        admitted/done times (seconds from trace start) filled in."""
        jobs = sorted(jobs, key=lambda j: j.arrival)
        queue = collections.deque()
        free_slots = list(range(len(self.slots)))
        running = {}  # slot -> (event, jobs, bytes, workspace)
        i = 0
        t0 = time.perf_counter()
        while i < len(jobs) or queue or running:
            now = time.perf_counter() - t0
            while i < len(jobs) and jobs[i].arrival <= now:
                j = jobs[i]
                i += 1
                if not self.policy.fits_ever(j):
                    j.rejected = True
                    continue
                queue.append(j)
            for slot in list(running):
                ev, group, nbytes, ws, base = running[slot]
                if ev.query():
                    t = time.perf_counter() - t0
                    err = int(self.err_host[slot])
                    for j in group:
                        j.done = t
                        if err:
                            j.failed, j.error = True, err
                        if on_done is not None:
                            on_done(j)
                        # the output's arena block is reused from now on:
                        # kept outputs are copied out of it (outside the budget)
                        j.keys_out = j.keys_out.clone() if self.keep_outputs else None
                    self.used -= nbytes
                    self.arena.release(base, nbytes)
                    del running[slot]
                    free_slots.append(slot)
            while free_slots and queue:
                group = self.policy.pick(queue, self.policy.budget - self.used)
                if not group:
                    break
                nbytes = sum(Arena.round(self._job_bytes(j)) for j in group)
                if len(group) > 1:
                    nbytes += Arena.round(self._batch_overhead(group))
                base = self.arena.alloc(nbytes)
                if base is None:
                    break  # free bytes are split into smaller blocks: wait for completions
                for _ in group:
                    queue.popleft()
                t = time.perf_counter() - t0
                for j in group:
                    j.admitted = t
                    j.nbytes = nbytes
                slot = free_slots.pop()
                ev, ws = self._launch(group, self.slots[slot], slot, base)
                running[slot] = (ev, group, nbytes, ws, base)
                self.used += nbytes
                self.peak_used = max(self.peak_used, self.used)
                self.max_in_flight = max(self.max_in_flight, len(running))
            if poll_sleep:
                time.sleep(poll_sleep)
        torch.cuda.synchronize(self.device)
        return jobs


def served_stats(jobs):
    """Latency percentiles (ms) and throughput of the jobs that completed
    without a device error: p50/p99 over all of them and over the first and
    second half by arrival (a stable queue keeps the two halves alike)."""
    ok = [j for j in jobs if j.done is not None and not j.failed]
    if not ok:
        return {"jobs": 0}
    lat = [j.latency * 1e3 for j in ok]
    half = len(ok) // 2
    span = max(j.done for j in ok) - min(j.arrival for j in ok)
    return {"p50_ms": round(percentile(lat, 50), 3), "p99_ms": round(percentile(lat, 99), 3),
            "p99_first_half_ms": round(percentile(lat[:half], 99), 3) if half else None,
            "p99_second_half_ms": round(percentile(lat[half:], 99), 3),
            "gkeys_s": round(sum(j.n for j in ok) / span / 1e9, 3) if span > 0 else None,
            "jobs": len(ok), "failed": sum(1 for j in jobs if j.failed),
            "rejected": sum(1 for j in jobs if j.rejected)}


def make_trace(count, seed, lam, log2_min=10, log2_max=28, widths=(16, 32, 64)):
    """Poisson arrivals at rate `lam` jobs/s of `count` jobs: n = floor(2^(a
    + (b-a) u)), width uniform over `widths`, distribution uniform over the
    ones valid for the width; every draw from the seeded counter generator."""
    import numpy as np
    import fsgen
    u = (fsgen.rand64(seed, 11, 0, count) >> np.uint64(11)).astype(np.float64) * 2.0 ** -53
    w = fsgen.rand64(seed, 12, 0, count)
    dsel = fsgen.rand64(seed, 13, 0, count)
    ua = (fsgen.rand64(seed, 14, 0, count) >> np.uint64(11)).astype(np.float64) * 2.0 ** -53
    gaps = -np.log(np.maximum(1.0 - ua, 2.0 ** -53)) / lam
    arrivals = np.cumsum(gaps) - gaps[0]
    jobs = []
    for k in range(count):
        n = int(np.floor(2.0 ** (log2_min + (log2_max - log2_min) * u[k])))
        bits = widths[int(w[k] % np.uint64(len(widths)))]
        dists = [d for d in fsgen.valid_dists(bits) if d not in ("presorted", "reverse")]
        dist = dists[int(dsel[k] % np.uint64(len(dists)))]
        jobs.append(Job(k, bits, n, dist, fsgen.seed_for(4, 0) + k, arrivals[k]))
    return jobs


def percentile(values, q):
    import numpy as np
    return float(np.percentile(np.asarray(values, dtype=np.float64), q)) if len(values) else None
