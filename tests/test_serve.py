"""Serving loop: admission policy on the CPU; the full server on the GPU
(each job's result equals the oracle's sort of that job alone, the memory
budget is never exceeded, work overlaps, oversized jobs are rejected)."""
import collections

import numpy as np
import pytest

from paper_2605_10390_amd.serve import AdmissionPolicy, Job, served_stats


def fake(jid, n, arrival=0.0, bits=32):
    return Job(jid, bits, n, "uniform", jid, arrival)


def test_policy_merges_small_jobs_in_arrival_order():
    p = AdmissionPolicy(10 ** 9, cost=lambda j: j.n, small_keys=100)
    q = collections.deque([fake(0, 10), fake(1, 20), fake(2, 1000), fake(3, 5)])
    assert [j.id for j in p.pick(q, 10 ** 9)] == [0, 1]
    q = collections.deque([fake(2, 1000), fake(3, 5)])
    assert [j.id for j in p.pick(q, 10 ** 9)] == [2]


def test_policy_waits_for_memory_and_rejects_impossible_jobs():
    p = AdmissionPolicy(5000, cost=lambda j: 4 * j.n, small_keys=100)
    big = fake(0, 1000)  # 4000 bytes: fits the budget, not the free memory below
    assert p.pick(collections.deque([big]), 3000) == []
    assert p.pick(collections.deque([big]), 4000) == [big]
    assert not p.fits_ever(fake(1, 2000))  # 8000 bytes > budget: rejected, never queued


def test_policy_batch_limits():
    p = AdmissionPolicy(10 ** 9, cost=lambda j: j.n, small_keys=100, batch_jobs=3, batch_keys=150)
    q = collections.deque([fake(i, 40) for i in range(6)])
    g = p.pick(q, 10 ** 9)
    assert [j.id for j in g] == [0, 1, 2]          # job limit
    p2 = AdmissionPolicy(10 ** 9, cost=lambda j: j.n, small_keys=100, batch_jobs=10, batch_keys=90)
    assert [j.id for j in p2.pick(q, 10 ** 9)] == [0, 1]  # key limit
    p3 = AdmissionPolicy(10 ** 9, cost=lambda j: j.n, small_keys=100)
    assert [j.id for j in p3.pick(q, 85)] == [0, 1]      # memory limit


def test_stats_leave_out_failed_and_rejected_jobs():
    jobs = [fake(i, 10, arrival=0.01 * i) for i in range(6)]
    for i, j in enumerate(jobs):
        j.done = j.arrival + 0.001 * (i + 1)
    jobs[2].failed, jobs[2].error = True, 4
    jobs[5].done, jobs[5].rejected = None, True
    st = served_stats(jobs)
    assert st["jobs"] == 4 and st["failed"] == 1 and st["rejected"] == 1
    assert st["p99_ms"] <= 5.0 + 1e-9  # job 2 (3 ms) is out; jobs 0,1,3,4: 1,2,4,5 ms
    assert abs(st["p50_ms"] - 3.0) < 1e-9


def test_arena_first_fit_and_merging():
    from paper_2605_10390_amd.serve import Arena
    a = Arena(4096, "cpu")
    x, y, z = a.alloc(1000), a.alloc(256), a.alloc(1024)
    assert (x, y, z) == (0, 1024, 1280)          # 256-byte blocks, first fit
    assert a.alloc(2048) is None                  # 1792 bytes left
    a.release(y, 256)
    assert a.alloc(512) == 2304                   # the 256-byte hole is too small
    a.release(x, 1000)                            # merges with the hole at 1024
    assert a.free[0] == (0, 1280)
    a.release(z, 1024)
    a.release(2304, 512)
    assert a.free == [(0, 4096)]                  # everything merged back


def attach_inputs(jobs, dev):
    """Each job's keys, resident on the device before the trace starts."""
    import fsgen
    for j in jobs:
        j.keys_in = fsgen.keys_device(j.dist, j.key_bits, j.n, j.seed, device=dev)


@pytest.mark.gpu
def test_server_results_alone_and_in_the_mix(gpu):
    import torch
    import fsgen
    import oracle
    from paper_2605_10390_amd.serve import SortServer, make_trace
    jobs = make_trace(48, fsgen.seed_for(4, 1), lam=1e5, log2_min=6, log2_max=20)
    got = {}

    def keep(j):
        got[j.id] = j.keys_out.cpu().numpy()

    attach_inputs(jobs, gpu)
    srv = SortServer(gpu, budget_bytes=2 << 30, slots=4, small_keys=1 << 14, keep_outputs=True)
    done = srv.serve(jobs, on_done=keep)
    assert all(j.done is not None and not j.failed for j in done)
    assert srv.peak_used <= 2 << 30
    assert srv.max_in_flight >= 2, "no two jobs ever ran at once"
    assert any(j.batched for j in done), "no small jobs were merged"
    for j in done:
        k = fsgen.keys_host(j.dist, j.key_bits, j.n, j.seed)
        assert np.array_equal(got[j.id], oracle.sort(k)), (j.id, j.key_bits, j.n, j.dist)


@pytest.mark.gpu
def test_server_budget_rejects_and_queues(gpu):
    import fsgen
    from paper_2605_10390_amd.serve import SortServer, make_trace
    jobs = make_trace(12, fsgen.seed_for(4, 2), lam=1e6, log2_min=12, log2_max=18)
    big = Job(99, 64, 1 << 24, "uniform", 5, 0.0)  # needs far more than the budget
    attach_inputs(jobs, gpu)
    srv = SortServer(gpu, budget_bytes=48 << 20, slots=3, small_keys=1 << 13)
    done = srv.serve(jobs + [big])
    assert big.rejected and big.done is None
    assert all(j.done is not None and not j.failed for j in done if j is not big)
    assert srv.peak_used <= 48 << 20
