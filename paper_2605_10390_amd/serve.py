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
    the queue.

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
                 "rejected", "keys_in", "keys_out", "nbytes")

    def __init__(self, jid, key_bits, n, dist, seed, arrival):
        self.id, self.key_bits, self.n, self.dist, self.seed = jid, key_bits, int(n), dist, seed
        self.arrival = float(arrival)
        self.admitted = self.done = None
        self.batched = False
        self.rejected = False
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


class SortServer:
    """Serves a trace of Jobs on one GPU with `slots` concurrent streams."""

    def __init__(self, device="cuda", budget_bytes=200 << 30, slots=4, small_keys=1 << 20,
                 batch_jobs=64, batch_keys=1 << 24, keep_outputs=False):
        self.device = torch.device(device)
        self.slots = [torch.cuda.Stream(self.device) for _ in range(slots)]  # default priority
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
    def _make_input(self, job):
        import fsgen
        job.keys_in = fsgen.keys_device(job.dist, job.key_bits, job.n, job.seed, device=self.device)
        job.keys_out = torch.empty_like(job.keys_in)

    def _launch(self, jobs, stream):
        with torch.cuda.stream(stream):
            for j in jobs:
                self._make_input(j)
            ws = Workspace(self.device)
            if len(jobs) == 1 and not jobs[0].batched:
                sort_keys(jobs[0].keys_in, out=jobs[0].keys_out, workspace=ws)
            else:
                for j in jobs:
                    j.batched = True
                SegmentBatch([(j.keys_in, j.keys_out, None, None) for j in jobs],
                             device=self.device).run(ws, stream=stream)
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
                ev, group, nbytes, ws = running[slot]
                if ev.query():
                    t = time.perf_counter() - t0
                    for j in group:
                        j.done = t
                        if on_done is not None:
                            on_done(j)
                        if not self.keep_outputs:
                            j.keys_in = j.keys_out = None
                    self.used -= nbytes
                    del running[slot]
                    free_slots.append(slot)
            while free_slots and queue:
                group = self.policy.pick(queue, self.policy.budget - self.used)
                if not group:
                    break
                for _ in group:
                    queue.popleft()
                nbytes = sum(self._job_bytes(j) for j in group)
                if len(group) > 1:
                    nbytes += self._batch_overhead(group)
                t = time.perf_counter() - t0
                for j in group:
                    j.admitted = t
                    j.nbytes = nbytes
                slot = free_slots.pop()
                ev, ws = self._launch(group, self.slots[slot])
                running[slot] = (ev, group, nbytes, ws)
                self.used += nbytes
                self.peak_used = max(self.peak_used, self.used)
                self.max_in_flight = max(self.max_in_flight, len(running))
            if poll_sleep:
                time.sleep(poll_sleep)
        torch.cuda.synchronize(self.device)
        return jobs


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
