"""Benchmark: Gkeys/s and fraction of the HBM roofline on one MI355X.

Default workload: 2^31 uint16 keys (4 GiB) with a uint32 payload equal to
the original index, keys i.i.d. uniform from the seeded generator; one
"step" is one complete stable sort of that batch (compressed histogram,
prefix scans and plan, two 8-bit scatter passes).  Inputs are resident in
HBM before timing starts.

Prints ONE JSON line.  Besides the contract fields it carries
  roofline      -- the dominant kernel (the scatter pass): algorithmic bytes
                   per launch / its average event-timed launch duration,
                   against the 8 TB/s HBM peak; `traffic` from the committed
                   rocprofv3 counter summary when it still matches the kernel
                   source, else null;
  cpu_baseline  -- the CPU oracle on a bounded sample of the same workload,
                   on this host's cores (and on one thread beside it);
  kernels       -- per-kernel-kind launches, average ms and GB/s.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload c1]
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Gkeys/s & % of HBM peak (16-bit, 4 GB); batched vs one-launch-per-sort"
HBM_PEAK_GBPS = 8000.0
PMC_SUMMARY = os.path.join(ROOT, "profiles", "scatter_u16u32_uniform_2e31_pmc.json")
KERNEL_SOURCES = ["paper_2605_10390_amd/csrc/tiled.hip", "paper_2605_10390_amd/csrc/fs_device.hpp"]
DOMINANT = {"c1": "k_tile_scatter", "c0": "k_expand16", "c2a": "k_tile_scatter", "c2b": "k_tile_scatter"}
COPY_PROBE_BYTES = 4 << 30

WORKLOADS = {
    # name: (key_bits, val_bytes, log2 n, distribution, description)
    "c1": (16, 4, 31, "uniform",
           "key-value sort of 2^31 uint16 keys (4 GiB) + uint32 index payload, uniform"),
    "c0": (16, 0, 28, "uniform", "keys-only sort of 2^28 uint16 keys (512 MiB), uniform"),
    "c2a": (32, 4, 31, "uniform", "key-value sort of 2^31 uint32 keys (8 GiB) + uint32 index, uniform"),
    "c2b": (64, 0, 32, "uniform", "keys-only sort of 2^32 uint64 keys (32 GiB), uniform"),
}


def kernel_source_hash():
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def scatter_bytes_per_key(key_bits, val_bytes):
    """Algorithmic bytes one scatter pass moves per key: read and write the
    key and its payload once."""
    return 2 * (key_bits // 8 + val_bytes)


def active_digits(keys, key_bits):
    """Which 8-bit digits are not trivial (not shared by every key); the sort
    skips the trivial ones on the device, so only these passes move data."""
    import torch
    kk = keys.view({16: torch.int16, 32: torch.int32, 64: torch.int64}[key_bits])
    out = []
    for j in range(key_bits // 8):
        d = (kk >> (8 * j)) & 0xFF
        out.append(bool(d.min() != d.max()))
    return out


PLAN_BYTE, PLAN_WORDS, PLAN_TRIE = 256, 72, 66  # the plan follows the workspace's error-word block


def plan_passes(ws):
    """The pass slots the device's plan ran (slot j sorted digit
    plan[4j+3]) and whether it took the sparse-trie window (plus fixup)."""
    import torch
    p = ws.buf[PLAN_BYTE:PLAN_BYTE + PLAN_WORDS * 4].view(torch.int32).cpu().tolist()
    slots = [j for j in range(16) if p[4 * j]]
    return slots, bool(p[PLAN_TRIE])


def scatter_pass_bytes(key_bits, val_bytes, active):
    """Algorithmic bytes per key of every scatter pass that runs.  A 16-bit
    pair sort's first pass writes, of each key, only the high byte the second
    pass sorts by (nothing when it is the only pass); the second pass reads
    that byte and writes only the payloads, the sorted keys being expanded
    from the 16-bit histogram."""
    kb, full = key_bits // 8, scatter_bytes_per_key(key_bits, val_bytes)
    if key_bits == 16 and val_bytes:
        out = []
        if active[0]:
            out.append(kb + val_bytes + (1 if active[1] else 0) + val_bytes)
        if active[1]:
            out.append(1 + 2 * val_bytes)
        return out
    return [full for a in active if a]


def algorithmic_bytes_per_key(key_bits, val_bytes, active):
    """Whole sort: one read of the keys for the histograms, then every pass
    that runs reads and writes key + payload; a 16-bit keys-only sort is one
    read plus one write of the keys (expansion), 16-bit pairs as in
    scatter_pass_bytes plus that expansion.  With no pass to run, the sort is
    the histogram read plus a copy."""
    kb = key_bits // 8
    if key_bits == 16 and val_bytes == 0:
        return 2 * kb
    if key_bits == 16:
        # histogram read, the passes, the expansion's key write; the payload
        # copy when no pass runs; the high-byte copy (read 2, write 1) when
        # only the second pass runs
        passes = scatter_pass_bytes(key_bits, val_bytes, active)
        extra = 2 * val_bytes if not passes else (kb + 1 if active[1] and not active[0] else 0)
        return kb + sum(passes) + kb + extra
    passes = sum(active)
    if passes == 0:
        return kb + 2 * (kb + val_bytes)
    return kb + passes * scatter_bytes_per_key(key_bits, val_bytes)


def read_traffic(source_hash):
    """HBM bytes per scatter launch from the committed counter summary, or
    None when absent or taken on a different kernel source."""
    try:
        with open(PMC_SUMMARY) as f:
            s = json.load(f)
    except (OSError, ValueError):
        return None
    if s.get("kernel_source_sha256_16") != source_hash:
        return None
    return s.get("hbm_bytes_per_launch")


def cpu_baseline(keys_dev, vals_dev, key_bits, val_bytes, budget_s=12.0):
    """The oracle as it stands on a bounded sample of the workload: the first
    2^26 keys (and payloads), sorted repeatedly for about budget_s / 2
    seconds single-threaded and as long split over the host's cores
    (oracle.sort_mt; the thread count is this process's CPU share).  `value` is the all-core rate; the paper's T_unit =
    n / (t * n_c) is given for both."""
    import numpy as np
    import oracle
    ns = min(1 << 26, keys_dev.numel())
    k = keys_dev[:ns].cpu().numpy()
    v = vals_dev[:ns].cpu().numpy() if vals_dev is not None else None
    oracle.load()
    # this process's CPU share: its affinity, capped by OMP_NUM_THREADS (16 if unset)
    share = int(os.environ.get("OMP_NUM_THREADS", "16") or 16)
    threads = max(1, min(len(os.sched_getaffinity(0)), share, 64))

    def timed(fn):
        reps, elapsed = 0, 0.0
        while elapsed < budget_s / 2 or reps == 0:
            t0 = time.perf_counter()
            fn()
            elapsed += time.perf_counter() - t0
            reps += 1
        return ns * reps / elapsed, reps, elapsed

    one, reps1, el1 = timed(lambda: oracle.sort(k) if v is None else oracle.sort(k, v))
    many, repsm, elm = timed(lambda: oracle.sort_mt(k, threads=threads) if v is None
                             else oracle.sort_mt(k, v, threads=threads))
    del np
    what = "keys only" if v is None else "with payload"
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            model = next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")), model)
    except OSError:
        pass
    return {"value": many / 1e9, "unit": "Gkeys/s", "cores": threads, "kind": "oracle",
            "sample": f"first 2^26 keys of the workload ({what}), sorted by the C oracle {repsm}x over "
                      f"{threads} threads ({elm:.1f} s) and {reps1}x on one thread ({el1:.1f} s)",
            "single_thread": {"value": one / 1e9, "unit": "Gkeys/s", "cores": 1},
            "host_cpu": model, "host_cpus_visible": os.cpu_count(), "host": host_cpu_description(),
            "t_unit_keys_per_s_per_core": {"all_cores": many / threads, "one_core": one}}


def build_c3(dev, count=100000, seed=None):
    """The batched workload: `count` segments with log-normal lengths
    (median 2048, sigma 2, capped at 2^22), 16-bit keys for even and 32-bit
    for odd segments, uniform or Zipf by a seeded coin, keys only.  Keys of
    each width class come from one device-generated array per distribution;
    segments are consecutive slices of it."""
    import numpy as np
    import torch
    import fsgen
    import paper_2605_10390_amd as fs
    seed = fsgen.seed_for(3, 0) if seed is None else seed
    L, bits, dist = fsgen.segment_plan(count, seed)
    pools = {}
    desc = np.zeros(count, dtype=fs.SEGMENT_DTYPE)
    keep = []
    for b in (16, 32):
        for dname in ("uniform", "zipf"):
            sel = np.flatnonzero((bits == b) & (dist == dname))
            tot = int(L[sel].sum())
            if tot == 0:
                continue
            # Zipf is drawn over 65536 ranks (16-bit values) for either width
            g = fsgen.keys_device(dname, b if dname == "uniform" else 16, tot,
                                  seed + b + (dname == "zipf"), device=dev)
            if b == 32 and dname == "zipf":
                g = g.to(torch.int32).view(torch.uint32)  # Zipf ranks as 32-bit keys
            out = torch.empty_like(g)
            keep += [g, out]
            esz = b // 8
            offs = np.concatenate([[0], np.cumsum(L[sel])[:-1]]).astype(np.uint64)
            desc["keys_in"][sel] = np.uint64(g.data_ptr()) + offs * np.uint64(esz)
            desc["keys_out"][sel] = np.uint64(out.data_ptr()) + offs * np.uint64(esz)
            desc["n"][sel] = L[sel].astype(np.uint64)
            desc["key_bits"][sel] = b
            pools[(b, dname)] = (g, out, sel, offs)
    batch = fs.SegmentBatch.from_array(desc, int(L.sum()), int(L.max()), device=dev, keep=keep)
    return batch, desc, pools, L


def segment_active_digits(pool, lengths, key_bits):
    """Per segment of `pool` (consecutive segments of the given lengths):
    how many 8-bit digits are not shared by all of its keys (the digits its
    sort runs passes for).  Plain PyTorch reductions over each digit's
    values (exact in float32: they are below 256)."""
    import numpy as np
    import torch
    lens = torch.from_numpy(np.asarray(lengths, dtype=np.int64)).to(pool.device)
    kk = pool.view({16: torch.int16, 32: torch.int32, 64: torch.int64}[key_bits])
    active = torch.zeros(lens.numel(), dtype=torch.int32, device=pool.device)
    for j in range(key_bits // 8):
        d = ((kk >> (8 * j)) & 0xFF).to(torch.float32)
        hi = torch.segment_reduce(d, "max", lengths=lens)
        lo = torch.segment_reduce(d, "min", lengths=lens)
        active += (hi != lo).to(torch.int32)
        del d, hi, lo
    return active.cpu().numpy()


def c3_algorithmic_bytes(desc, L, pools, tuning):
    """Algorithmic bytes of one C3 step, per bin, from the bins the
    classifier picks under `tuning` (segments of at most 64 keys: wave bin;
    16-bit keys from expand16_min_keys: the 16-bit-digit bin; what fits the
    LDS bin's bound and 32 KiB; the rest, one workgroup or the large bin):
      wave and LDS bins   read and write each key once: 2k
      16-bit-digit bin    histogram read 2 + expansion write 2
      one-WG / large bin  digit histograms k + 2k per active digit (a
                          segment with no active digit is copied: 2k)."""
    import numpy as np
    kb = desc["key_bits"].astype(np.int64) // 8
    n = L.astype(np.int64)
    smax = np.array(list(tuning.small_max_keys), dtype=np.int64)
    small_max = np.where(kb == 2, smax[0], np.where(kb == 4, smax[1], smax[2]))
    small_cap = (32768 - 16) // kb
    wave = n <= 64
    expand = ~wave & (kb == 2) & (n >= int(tuning.expand16_min_keys))
    small = ~wave & ~expand & (n <= np.minimum(small_cap, small_max))
    rest = ~(wave | expand | small)
    active = np.zeros(n.size, dtype=np.int64)
    for (b, dname), (g, out, sel, offs) in pools.items():
        active[sel] = segment_active_digits(g, L[sel], b)
    rest_bytes = np.where(active > 0, kb * n + 2 * kb * n * active, kb * n + 2 * kb * n)
    wg = rest & (n <= int(tuning.large_wg_max_keys))
    out = {"wave": int((2 * kb * n)[wave].sum()), "lds": int((2 * kb * n)[small].sum()),
           "digit16": int((4 * n)[expand].sum()), "one_workgroup": int(rest_bytes[wg].sum()),
           "large": int(rest_bytes[rest & ~wg].sum())}
    keys = {"wave": int(n[wave].sum()), "lds": int(n[small].sum()), "digit16": int(n[expand].sum()),
            "one_workgroup": int(n[wg].sum()), "large": int(n[rest & ~wg].sum())}
    return out, keys


def oracle_sample_rate(items, budget_s=12.0, threads=None, seed=0, one_at_a_time=False):
    """The oracle timed on a bounded sample: `items` is a list of (n, fetch)
    where fetch() returns the host keys of one independent sort (a segment
    or a job).  Items are drawn with probability proportional to n (so the
    rate is weighted like the whole batch's keys) and sorted until about
    budget_s of sorting time: one per thread by oracle.sort, or with
    one_at_a_time each by oracle.sort_mt over all the threads.  Only the
    sorts are timed.  Returns (keys/s, sampled keys, sorts, sorting
    seconds, threads)."""
    import numpy as np
    from concurrent.futures import ThreadPoolExecutor
    import oracle
    oracle.load()
    share = int(os.environ.get("OMP_NUM_THREADS", "16") or 16)
    threads = threads or max(1, min(len(os.sched_getaffinity(0)), share, 64))
    rng = np.random.default_rng(seed)
    w = np.array([float(it[0]) for it in items])
    order = rng.choice(len(items), size=min(len(items), 4096), replace=False, p=w / w.sum())
    done_keys = sorts = 0
    wall = 0.0
    step = 1 if one_at_a_time else threads
    with ThreadPoolExecutor(threads) as ex:
        pos = 0
        while pos < len(order) and wall < budget_s:
            batch = [items[i][1]() for i in order[pos:pos + step]]
            pos += step
            t0 = time.perf_counter()
            if one_at_a_time:
                oracle.sort_mt(batch[0], threads=threads)
            else:
                list(ex.map(oracle.sort, batch))
            wall += time.perf_counter() - t0
            done_keys += sum(int(b.size) for b in batch)
            sorts += len(batch)
    return done_keys / wall, done_keys, sorts, wall, threads


def host_cpu_description():
    """lscpu's model, sockets, cores per socket and threads (or /proc/cpuinfo's model)."""
    import subprocess
    info = {}
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for ln in out.splitlines():
            k, _, v = ln.partition(":")
            info[k.strip()] = v.strip()
    except (OSError, subprocess.SubprocessError):
        pass
    model = info.get("Model name")
    if not model:
        try:
            with open("/proc/cpuinfo") as f:
                model = next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")), None)
        except OSError:
            model = None
    return {"model": model or "unknown", "sockets": info.get("Socket(s)"),
            "cores_per_socket": info.get("Core(s) per socket"), "threads": info.get("CPU(s)"),
            "process_cpu_share": len(os.sched_getaffinity(0))}


def run_c3(args):
    import ctypes
    import numpy as np
    import torch
    import oracle
    import paper_2605_10390_amd as fs
    dev = torch.device("cuda:0")
    batch, desc, pools, L = build_c3(dev)
    n = batch.total_keys
    ws = fs.Workspace(dev)
    ws.get(batch.workspace_bytes())
    tuned, tune_info = None, None
    if not args.no_autotune:
        # launch tuning chosen on this batch before anything is timed
        from paper_2605_10390_amd import autotune
        t0 = time.perf_counter()
        tuned, rep = autotune.tune_batch(batch, ws, reps=3, sweeps=2,
                                         log=lambda m: print(m, file=sys.stderr, flush=True))
        tune_info = {"tuning": tuned.as_dict(), "start_ms": round(rep["start_ms"], 4),
                     "tuned_ms": round(rep["best_ms"], 4), "measured": rep["measured"],
                     "seconds": round(time.perf_counter() - t0, 1)}
    graph = fs.CapturedSort(lambda: batch.run(ws, tuning=tuned), dev)
    for _ in range(args.warmup):
        graph.replay()
    torch.cuda.synchronize()
    print(f"[bench] c3: {batch.count} segments, {n} keys; warmup done", file=sys.stderr, flush=True)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(args.steps):
        graph.replay()
    e1.record()
    torch.cuda.synchronize()
    ms_batched = e0.elapsed_time(e1) / args.steps
    if ws.error_word() != 0:
        raise SystemExit(f"device error word {ws.error_word():#x}")
    # spot check: sampled segments against the oracle
    rng = np.random.default_rng(0)
    for i in rng.choice(batch.count, size=24, replace=False):
        b = int(desc["key_bits"][i])
        for (pb, dname), (g, out, sel, offs) in pools.items():
            if pb != b:
                continue
            pos = np.searchsorted(sel, i)
            if pos < len(sel) and sel[pos] == i:
                o, m = int(offs[pos]), int(L[i])
                assert np.array_equal(out[o:o + m].cpu().numpy(), oracle.sort(g[o:o + m].cpu().numpy())), i
    gk = n / (ms_batched / 1e3) / 1e9
    out = {
        "metric": METRIC, "value": round(gk, 3), "unit": "Gkeys/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_batched, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u16/u32 mixed", "data": "synthetic",
        "config": {"workload": f"batched segmented sort: {batch.count} segments, log-normal lengths "
                               "(median 2048, sigma 2, cap 2^22), half u16 half u32, uniform/Zipf, keys only",
                   "n": n, "segments": batch.count, "max_segment": int(L.max()),
                   "parallelism": "single GPU", "graph": True},
    }
    out["autotune"] = tune_info
    tuning_used = tuned if tuned is not None else fs.get_tuning()
    by_bin, keys_by_bin = c3_algorithmic_bytes(desc, L, pools, tuning_used)
    alg = sum(by_bin.values())
    achieved = alg / (ms_batched / 1e3) / 1e9
    out["roofline"] = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                       "frac": round(achieved / HBM_PEAK_GBPS, 4), "traffic": None,
                       "scope": "whole step (every segmented kernel of the graph): algorithmic bytes of "
                                "the bins the classifier picks, over the step time",
                       "bytes_per_step_by_bin": by_bin, "keys_by_bin": keys_by_bin}
    if not args.no_cpu_baseline:
        items = []
        for (b, dname), (g, outp, sel, offs) in pools.items():
            for i, o in zip(sel.tolist(), offs.tolist()):
                m = int(L[i])
                items.append((m, (lambda g=g, o=int(o), m=m: g[o:o + m].cpu().numpy())))
        rate, sk, sorts, wall, thr = oracle_sample_rate(items)
        out["cpu_baseline"] = {"value": round(rate / 1e9, 4), "unit": "Gkeys/s", "cores": thr, "kind": "oracle",
                               "sample": f"{sorts} segments ({sk} keys) drawn with probability proportional "
                                         f"to length, each sorted alone by the C oracle, {thr} at a time "
                                         f"({wall:.1f} s of sorting); the whole batch at this rate: "
                                         f"{n / rate:.1f} s",
                               "host_cpu": host_cpu_description()}
    if args.no_loop_baseline:
        print(json.dumps(out), flush=True)
        return
    # baseline: one fs_sort_keys call per segment from a host loop, no graphs
    Lb = fs.lib()
    st = ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)
    wsb = fs.Workspace(dev)
    need = max(fs.sort_keys_workspace_bytes(int(L.max()), 16), fs.sort_keys_workspace_bytes(int(L.max()), 32))
    buf = wsb.get(need)
    size = ctypes.c_size_t(buf.numel())
    bp = ctypes.c_void_p(buf.data_ptr())
    kin, kout, nn, kb = (desc["keys_in"].tolist(), desc["keys_out"].tolist(), desc["n"].tolist(),
                         desc["key_bits"].tolist())
    torch.cuda.synchronize()
    b0, b1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    b0.record()
    for i in range(batch.count):
        size.value = buf.numel()
        r = Lb.fs_sort_keys(ctypes.c_void_p(kin[i]), ctypes.c_void_p(kout[i]), nn[i], kb[i], 0, bp,
                            ctypes.byref(size), st)
        if r != 0:
            raise SystemExit(f"fs_sort_keys failed on segment {i}: {r}")
    b1.record()
    torch.cuda.synchronize()
    ms_loop = b0.elapsed_time(b1)
    out["one_launch_per_sort"] = {"ms": round(ms_loop, 3), "gkeys_s": round(n / (ms_loop / 1e3) / 1e9, 3),
                                  "calls": batch.count}
    out["batched_speedup"] = round(ms_loop / ms_batched, 2)
    print(json.dumps(out), flush=True)


def c4_pools(dev, seed, pool_keys=1 << 28):
    """Resident inputs of the served stream: one device array of 2^28 keys
    per (width, distribution) a job can draw; a job's input is a slice of
    its pool, so every input is in HBM before the trace starts."""
    import fsgen
    pools = {}
    for bits in (16, 32, 64):
        for di, dist in enumerate(fsgen.valid_dists(bits)):
            if dist in ("presorted", "reverse"):
                continue
            pools[(bits, dist)] = fsgen.keys_device(dist, bits, pool_keys, seed + 64 * bits + di, device=dev)
    return pools


def attach_pool_inputs(jobs, pools):
    for j in jobs:
        g = pools[(j.key_bits, j.dist)]
        off = ((j.seed * 0x9E3779B97F4A7C15) >> 11) % (g.numel() - j.n + 1)
        j.keys_in = g[off:off + j.n]


def run_c4(args):
    """Served stream: Poisson arrivals of sort jobs (sizes log-uniform
    2^10..2^28 keys, widths 16/32/64, mixed distributions), 200 GB device
    budget, continuous batching over 4 streams, against FIFO one job at a
    time.  A seeded prefix of `args.jobs` jobs of the 20k-job stream is
    served.  Every input is resident in HBM before any timing (slices of
    per-distribution pools).  Capacity = the prefix's keys over its
    makespan when every job arrives at once; the arrival rate is then rho
    times the continuous-batching capacity, rho = 0.5 and 0.9, and both
    servers are run on each trace."""
    import numpy as np
    import torch
    import fsgen
    from paper_2605_10390_amd.serve import SortServer, make_trace, served_stats
    dev = torch.device("cuda:0")
    seed = fsgen.seed_for(4, 0)
    budget = 200 << 30
    pools = c4_pools(dev, seed + 7)
    torch.cuda.synchronize()
    torch.cuda.reset_peak_memory_stats(dev)
    modes = (("continuous_batching", dict(slots=4)), ("fifo_one_at_a_time", dict(slots=1, small_keys=0)))

    def serve(lam, kw):
        trace = make_trace(args.jobs, seed, lam=lam)
        attach_pool_inputs(trace, pools)
        srv = SortServer(dev, budget_bytes=budget, **kw)
        t0 = time.perf_counter()
        done = srv.serve(trace)
        wall = time.perf_counter() - t0
        st = served_stats(done)
        st.update({"launches": srv.launches, "peak_budgeted_gb": round(srv.peak_used / 2 ** 30, 2),
                   "max_in_flight": srv.max_in_flight, "wall_s": round(wall, 2)})
        for j in trace:
            j.keys_in = None
        del srv
        return done, st

    warm = make_trace(48, seed + 1, lam=1e9)
    attach_pool_inputs(warm, pools)
    SortServer(dev, budget_bytes=budget, slots=4).serve(warm)  # module loads, the arena's allocation
    mean_n = float(np.mean([j.n for j in make_trace(args.jobs, seed, lam=1.0)]))
    capacity = {}
    for name, kw in modes:
        done, st = serve(1e12, kw)  # every job arrives at t = 0
        ok = [j for j in done if j.done is not None and not j.failed]
        capacity[name] = {"gkeys_s": round(sum(j.n for j in ok) / max(j.done for j in ok) / 1e9, 3),
                          "failed": st["failed"], "wall_s": st["wall_s"]}
        print(f"[bench] c4 capacity {name}: {capacity[name]}", file=sys.stderr, flush=True)
    cap = capacity["continuous_batching"]["gkeys_s"] * 1e9
    served = {}
    for rho in (0.5, 0.9):
        lam = rho * cap / mean_n
        served[f"rho_{rho}"] = {"lambda_jobs_s": round(lam, 3)}
        for name, kw in modes:
            _, st = serve(lam, kw)
            served[f"rho_{rho}"][name] = st
            print(f"[bench] c4 rho {rho} {name}: {st}", file=sys.stderr, flush=True)
    reserved = torch.cuda.max_memory_reserved(dev)
    failed = sum(capacity[m]["failed"] for m in capacity) + sum(
        served[r][m].get("failed", 0) for r in served for m, _ in modes)
    if failed:
        raise SystemExit(f"{failed} served jobs reported a device error")
    out = {"metric": METRIC, "value": capacity["continuous_batching"]["gkeys_s"], "unit": "Gkeys/s",
           "n_gpus": 1, "steps": 1, "warmup": 0, "ms_per_step": None, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "u16/u32/u64 mixed", "data": "synthetic",
           "config": {"workload": f"served sort stream: seeded prefix of {args.jobs} of 20000 jobs, n log-uniform "
                                  "2^10..2^28, widths 16/32/64, mixed distributions, 200 GB budget, inputs "
                                  "resident before arrival; value = continuous-batching capacity (every job "
                                  "arriving at once); Poisson arrivals at rho = 0.5 and 0.9 of it",
                      "jobs": args.jobs, "mean_keys_per_job": round(mean_n, 1),
                      "parallelism": "single GPU, 4 streams"},
           "capacity": capacity,
           "batched_speedup": round(capacity["continuous_batching"]["gkeys_s"] /
                                    capacity["fifo_one_at_a_time"]["gkeys_s"], 3),
           "served": served,
           "device_memory": {"max_reserved_gb": round(reserved / 2 ** 30, 2),
                             "server_arena_gb": round(budget / 2 ** 30, 2),
                             "resident_input_pools_gb": round(sum(g.numel() * g.element_size()
                                                                  for g in pools.values()) / 2 ** 30, 2)}}
    if not args.no_cpu_baseline:
        jobs = make_trace(args.jobs, seed, lam=1.0)
        attach_pool_inputs(jobs, pools)
        items = [(j.n, (lambda j=j: j.keys_in.cpu().numpy())) for j in jobs]
        rate, sk, sorts, wall, thr = oracle_sample_rate(items, seed=4, one_at_a_time=True)
        total = sum(j.n for j in jobs)
        out["cpu_baseline"] = {"value": round(rate / 1e9, 4), "unit": "Gkeys/s", "cores": thr, "kind": "oracle",
                               "sample": f"{sorts} jobs of the prefix ({sk} keys) drawn with probability "
                                         f"proportional to size, each sorted alone by the C oracle split over "
                                         f"{thr} threads ({wall:.1f} s of sorting); the whole prefix at this "
                                         f"rate: {total / rate:.1f} s",
                               "host_cpu": host_cpu_description()}
    print(json.dumps(out), flush=True)


# the paper's comparison figures, each with the hardware it names (context,
# not targets; the paper reports no GPU or FPGA timings of its own method)
PAPER_CONTEXT = {
    "fractalsort_cpu_4gb_u16": "21.22 s for 4 GB of 16-bit keys (2^31 keys, 0.101 Gkeys/s) on a 4-core "
                               "i7-8665U, Numba (Sec. IV-E)",
    "paradis_cpu_4gb_u16": "4.6 s (0.467 Gkeys/s) on a 32-core Xeon E7-8837, quoted by the paper (Sec. IV-E)",
    "b_eff_ratios": "the paper's bandwidth-efficiency gain at 16 GB, p = 16 (Sec. IV-F): 6x over Paradis "
                    "(CPU), 3x over HRS (GPU), 2.5x over Bonsai (FPGA); b_eff here = algorithmic bytes / "
                    "(FETCH_SIZE + WRITE_SIZE) of the dominant kernel",
}

PCIE5_X16_GBPS = 63.0  # per direction: 32 GT/s x 16 lanes, 128b/130b coding


def run_stream16(args):
    """Batch stream sorting of 16-bit keys that live in host memory: 2^31
    uint16 keys (4 GiB, pinned), copied to the device 2^26 keys at a time,
    counted into one resident 2^16-bin histogram as they arrive and written
    back sorted through the same staging slots (fs_sort16_host).  The host
    link carries 2 B per key in and 2 B out, one direction after the other,
    so the bound is the link's per-direction rate; the plain pinned copy
    rates of both directions are measured beside it."""
    import torch
    import fsgen
    import paper_2605_10390_amd as fs
    dev = torch.device("cuda:0")
    n, batch = 1 << 31, 1 << 26
    seed = fsgen.seed_for(1, 0)
    src = torch.empty(n, dtype=torch.uint16, pin_memory=True)
    src.copy_(fsgen.keys_device("uniform", 16, n, seed, device=dev))
    out = torch.empty(n, dtype=torch.uint16, pin_memory=True)
    ws = fs.Workspace(dev)
    ws.get(fs.sort16_host_workspace_bytes(batch))
    xs = torch.cuda.Stream(dev)
    # plain pinned copies of the same 4 GiB, each direction alone
    d = torch.empty(n, dtype=torch.uint16, device=dev)
    rates = {}
    for name, (dst, srct) in (("h2d", (d, src)), ("d2h", (out, d))):
        dst.copy_(srct, non_blocking=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        dst.copy_(srct, non_blocking=True)
        torch.cuda.synchronize()
        rates[name] = 2 * n / (time.perf_counter() - t0) / 1e9
    del d
    for _ in range(args.warmup):
        fs.sort16_host(src, out=out, batch_keys=batch, workspace=ws, copy_stream=xs, device=dev)
    print(f"[bench] stream16 warmup done; pinned copy GB/s {rates}", file=sys.stderr, flush=True)
    times = []
    for _ in range(args.steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fs.sort16_host(src, out=out, batch_keys=batch, workspace=ws, copy_stream=xs, device=dev)
        times.append(time.perf_counter() - t0)  # the call returns with the host output complete
    ms = 1e3 * sum(times) / len(times)
    o = out.view(torch.int16)
    step = 1 << 28
    for a in range(0, n, step):  # cheap validity check outside the timed region
        c = o[a:a + step].to(torch.int32) & 0xFFFF
        assert bool((c[1:] >= c[:-1]).all()), "output not sorted"
    achieved = 4 * n / (ms / 1e3) / 1e9
    ideal_ms = 1e3 * (2 * n / (rates["h2d"] * 1e9) + 2 * n / (rates["d2h"] * 1e9))
    res = {"metric": "Gkeys/s, 16-bit keys sorted host to host through the device (batch stream)",
           "value": round(n / (ms / 1e3) / 1e9, 3), "unit": "Gkeys/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": round(ms, 3), "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "u16", "data": "synthetic",
           "config": {"workload": "batch stream sort of 2^31 uint16 keys (4 GiB) in pinned host memory, "
                                  "2^26-key batches, uniform", "n": n, "batch_keys": batch, "seed": seed,
                      "parallelism": "single GPU, copy stream + compute stream"},
           "roofline": {"bound": "pcie", "kernel": None, "achieved": round(achieved, 2),
                        "peak": PCIE5_X16_GBPS, "unit": "GB/s", "frac": round(achieved / PCIE5_X16_GBPS, 4),
                        "traffic": None, "bytes_per_key": 4},
           "pinned_copy_gbps": {k: round(v, 2) for k, v in rates.items()},
           "frac_of_measured_copies": round(ideal_ms / ms, 4)}
    if not args.no_cpu_baseline:
        print("[bench] timing the CPU oracle on a sample", file=sys.stderr, flush=True)
        res["cpu_baseline"] = cpu_baseline(src, None, 16, 0)
    print(json.dumps(res), flush=True)


def run_host32(args):
    """Out-of-core sort of 32-bit keys (fs_sort_host): 2^31 uint32 keys
    (8 GiB) in pinned host memory, with device ranges of at most 2^29 keys,
    so the sort spills through four or more ranges as if the keys did not fit
    the device.  The input crosses the host link (ranges + 2) times and the
    output once; the bound is the link's per-direction rate."""
    import torch
    import fsgen
    import paper_2605_10390_amd as fs
    dev = torch.device("cuda:0")
    n, batch, dk = 1 << 31, 1 << 26, 1 << 29
    seed = fsgen.seed_for(2, 0)
    src = torch.empty(n, dtype=torch.uint32, pin_memory=True)
    src.copy_(fsgen.keys_device("uniform", 32, n, seed, device=dev))
    out = torch.empty(n, dtype=torch.uint32, pin_memory=True)
    ws = fs.Workspace(dev)
    xs = torch.cuda.Stream(dev)
    for _ in range(args.warmup):
        fs.sort_host(src, out=out, batch_keys=batch, device_keys=dk, workspace=ws, copy_stream=xs, device=dev)
    times = []
    for _ in range(args.steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fs.sort_host(src, out=out, batch_keys=batch, device_keys=dk, workspace=ws, copy_stream=xs, device=dev)
        times.append(time.perf_counter() - t0)
    ms = 1e3 * sum(times) / len(times)
    o = out.view(torch.int32)
    for a in range(0, n, 1 << 28):  # cheap validity check outside the timed region
        c = o[a:a + (1 << 28)].to(torch.int64) & 0xFFFFFFFF
        assert bool((c[1:] >= c[:-1]).all()), "output not sorted"
    ranges = -(-n // dk)  # at least; uniform keys fill ranges nearly to the bound
    link_bytes = 4 * n * (ranges + 2) + 4 * n
    achieved = link_bytes / (ms / 1e3) / 1e9
    res = {"metric": "Gkeys/s, 32-bit keys sorted host to host through the device (out-of-core MSD spill)",
           "value": round(n / (ms / 1e3) / 1e9, 3), "unit": "Gkeys/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": round(ms, 3), "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "u32", "data": "synthetic",
           "config": {"workload": "out-of-core sort of 2^31 uint32 keys (8 GiB) in pinned host memory, device "
                                  "ranges of at most 2^29 keys, 2^26-key batches, uniform", "n": n,
                      "batch_keys": batch, "device_keys": dk, "seed": seed,
                      "parallelism": "single GPU, copy stream + compute stream"},
           "roofline": {"bound": "pcie", "kernel": None, "achieved": round(achieved, 2), "peak": PCIE5_X16_GBPS,
                        "unit": "GB/s", "frac": round(achieved / PCIE5_X16_GBPS, 4), "traffic": None,
                        "bytes_per_key": 4 * (ranges + 3)}}
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline(src, None, 32, 0)
    print(json.dumps(res), flush=True)


def _timed_with_kinds(step, steps):
    """Time `steps` calls of step() between two events on the current stream,
    with the library's per-kind launch timers on; returns (ms_total, kinds)."""
    import torch
    import ctypes
    import paper_2605_10390_amd as fs
    L = fs.lib()
    L.fs_profile_enable(1)
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0.record()
    for _ in range(steps):
        step()
    t1.record()
    torch.cuda.synchronize()
    kernels = {}
    for name, kid in {"histogram": 0, "plan": 1, "scatter": 2, "expand": 3, "aux": 4}.items():
        c, k, ms = ctypes.c_uint64(), ctypes.c_uint64(), ctypes.c_double()
        L.fs_profile_read(kid, ctypes.byref(c), ctypes.byref(k), ctypes.byref(ms))
        kernels[name] = {"launches": c.value, "keys": k.value, "ms_total": round(ms.value, 4)}
        if c.value:
            kernels[name]["ms_avg"] = round(ms.value / c.value, 4)
    L.fs_profile_enable(0)
    return t0.elapsed_time(t1), kernels


def _scatter_roofline(kernels, steps, bytes_per_launch, passes_per_step):
    """HBM roofline of the scatter passes: algorithmic bytes of the passes
    that run over the event-timed scatter time per step."""
    ms = kernels["scatter"]["ms_total"] / steps
    achieved = bytes_per_launch * passes_per_step / (ms / 1e3) / 1e9 if ms > 0 else None
    return {"bound": "hbm", "kernel": "k_tile_scatter", "achieved": round(achieved, 1) if achieved else None,
            "peak": HBM_PEAK_GBPS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBPS, 4) if achieved else None,
            "traffic": None}


def run_c8(args):
    """8-bit keys with a u32 index payload: 2^30 pairs, uniform keys (the
    high byte of the uniform 16-bit recipe).  The whole key is one digit:
    one tile-histogram read and one scatter pass of 2(1 + 4) bytes per key."""
    import torch
    import fsgen
    import paper_2605_10390_amd as fs
    dev = torch.device("cuda:0")
    n = 1 << 30
    seed = fsgen.seed_for(8, 0)
    k16 = fsgen.keys_device("uniform", 16, n, seed, device=dev)
    keys = ((k16.view(torch.int16).to(torch.int32) >> 8) & 0xFF).to(torch.uint8)
    del k16
    vals = fsgen.index_device(n, 4, device=dev)
    ko, vo = torch.empty_like(keys), torch.empty_like(vals)
    ws = fs.Workspace(dev)

    def step():
        fs.sort_pairs(keys, vals, keys_out=ko, vals_out=vo, workspace=ws)

    for _ in range(args.warmup):
        step()
    ms_total, kernels = _timed_with_kinds(step, args.steps)
    if ws.error_word() != 0:
        raise SystemExit(f"device error word {ws.error_word():#x}: result invalid")
    kk = ko.to(torch.int32)
    assert bool((kk[1:] >= kk[:-1]).all()), "output keys not sorted"
    assert torch.equal(keys[vo.view(torch.int32).to(torch.int64)], ko), "payload does not index the keys"
    ms = ms_total / args.steps
    res = {"metric": "Gkeys/s, 8-bit keys with a 32-bit index payload", "value": round(n / (ms / 1e3) / 1e9, 3),
           "unit": "Gkeys/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 4),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u8+u32",
           "data": "synthetic",
           "config": {"workload": "key-value sort of 2^30 uint8 keys + uint32 index payload, uniform", "n": n,
                      "key_bits": 8, "val_bytes": 4, "seed": seed, "parallelism": "single GPU"},
           "roofline": _scatter_roofline(kernels, args.steps, n * 10, 1),
           "hbm_frac_whole_sort": round(n * 11 / (ms / 1e3) / 1e9 / HBM_PEAK_GBPS, 4),
           "algorithmic_bytes_per_key": 11, "kernels": kernels}
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline(keys, vals, 8, 4)
    print(json.dumps(res), flush=True)


def run_wide128(args):
    """Keys of two 64-bit words (128 bits), keys only: 2^28 keys of uniform
    words.  Two rounds, least significant word first; each round gathers one
    word through the permutation and sorts (word, u32 permutation entry)
    pairs in 8 passes of 2(8 + 4) bytes per key; the last permutation moves
    the whole keys."""
    import torch
    import fsgen
    import paper_2605_10390_amd as fs
    dev = torch.device("cuda:0")
    n, words = 1 << 28, 2
    seed = fsgen.seed_for(9, 0)
    keys = fsgen.keys_device("uniform", 64, n * words, seed, device=dev).view(torch.int64).view(n, words)
    ko = torch.empty_like(keys)
    ws = fs.Workspace(dev)

    def step():
        fs.sort_wide(keys, keys_out=ko, workspace=ws)

    for _ in range(args.warmup):
        step()
    ms_total, kernels = _timed_with_kinds(step, args.steps)
    if ws.error_word() != 0:
        raise SystemExit(f"device error word {ws.error_word():#x}: result invalid")
    # sorted as unsigned 128-bit values: (hi, lo) non-decreasing
    hi = ko[:, 1] ^ (-(1 << 63))
    lo = ko[:, 0] ^ (-(1 << 63))
    ok = (hi[1:] > hi[:-1]) | ((hi[1:] == hi[:-1]) & (lo[1:] >= lo[:-1]))
    assert bool(ok.all()), "output keys not sorted"
    ms = ms_total / args.steps
    passes = 8 * words
    res = {"metric": "Gkeys/s, 128-bit keys (two 64-bit words), keys only", "value": round(n / (ms / 1e3) / 1e9, 3),
           "unit": "Gkeys/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 4),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u64x2",
           "data": "synthetic",
           "config": {"workload": "keys-only sort of 2^28 keys of 128 bits (4 GiB), uniform words", "n": n,
                      "key_words": words, "seed": seed, "parallelism": "single GPU"},
           "roofline": _scatter_roofline(kernels, args.steps, n * 24, passes), "kernels": kernels}
    print(json.dumps(res), flush=True)


def pmc_summary(fetch_csv, write_csv, kernel, out_path, command):
    """Turn two rocprofv3 --pmc runs (FETCH_SIZE, then WRITE_SIZE; KiB per
    dispatch) of `bench.py --copy-probe` into HBM bytes per launch of
    `kernel`.  Each counter is scaled by what it reads for the plain 4 GiB
    device copy the probe runs first (4 GiB read, 4 GiB written)."""
    import csv
    import collections

    def per_dispatch(path):
        acc = collections.OrderedDict()
        for r in csv.DictReader(open(path)):
            key = (int(r["Dispatch_Id"]), r["Kernel_Name"])
            acc[key] = acc.get(key, 0.0) + float(r["Counter_Value"])
        return acc

    f, w = per_dispatch(fetch_csv), per_dispatch(write_csv)
    copy_f = max(v for (d, k), v in f.items() if "copyBuffer" in k)
    copy_w = max(v for (d, k), v in w.items() if "copyBuffer" in k)
    ff, wf = COPY_PROBE_BYTES / (copy_f * 1024.0), COPY_PROBE_BYTES / (copy_w * 1024.0)
    kf = [v * 1024.0 * ff for (d, k), v in f.items() if kernel in k]
    kw = [v * 1024.0 * wf for (d, k), v in w.items() if kernel in k]
    summary = {"kernel": kernel, "launches": len(kf),
               "fetch_bytes_per_launch": sum(kf) / len(kf), "write_bytes_per_launch": sum(kw) / len(kw),
               "hbm_bytes_per_launch": (sum(kf) + sum(kw)) / len(kf),
               "fetch_scale": ff, "write_scale": wf,
               "calibration": "plain device copy of 4 GiB (rocclr copyBuffer) in the same run",
               "kernel_source_sha256_16": kernel_source_hash(), "command": command}
    with open(out_path, "w") as fo:
        json.dump(summary, fo, indent=1)
    print(json.dumps(summary))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="c1", choices=sorted(WORKLOADS) + ["c3", "c4", "stream16", "host32", "c8", "wide128"])
    ap.add_argument("--jobs", type=int, default=20000, help="served-stream prefix length (c4)")
    ap.add_argument("--dist", default=None,
                    help="c0/c1/c2a/c2b: key distribution (16-bit: uniform gaussian zipf equal presorted "
                         "reverse; wider: uniform small20 hot90); default uniform")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true", help="c3: default launch tuning")
    ap.add_argument("--no-loop-baseline", action="store_true",
                    help="c3: skip the one-call-per-segment comparison (for kernel profiles)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="run a plain 4 GiB device copy first (counter calibration)")
    ap.add_argument("--pmc-summary", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="summarise two rocprofv3 --pmc runs of this bench into profiles/")
    args = ap.parse_args()
    if args.pmc_summary:
        cmd = ("rocprofv3 --pmc FETCH_SIZE (then WRITE_SIZE) --output-format csv -- "
               f"python bench.py --workload {args.workload} --steps 1 --warmup 0 --no-cpu-baseline --copy-probe")
        return pmc_summary(args.pmc_summary[0], args.pmc_summary[1], DOMINANT[args.workload],
                           PMC_SUMMARY, cmd)
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(multi-GPU sharding is designed, not measured)", file=sys.stderr)
        sys.exit(2)

    if args.workload == "c3":
        return run_c3(args)
    if args.workload == "c4":
        return run_c4(args)
    if args.workload == "stream16":
        return run_stream16(args)
    if args.workload == "host32":
        return run_host32(args)
    if args.workload == "c8":
        return run_c8(args)
    if args.workload == "wide128":
        return run_wide128(args)

    import torch
    import ctypes
    import fsgen
    import paper_2605_10390_amd as fs

    key_bits, val_bytes, logn, dist, desc = WORKLOADS[args.workload]
    if args.dist is not None:
        if args.dist not in fsgen.valid_dists(key_bits):
            raise SystemExit(f"--dist {args.dist}: not a {key_bits}-bit distribution "
                             f"({', '.join(fsgen.valid_dists(key_bits))})")
        desc = desc.replace(f", {dist}", f", {args.dist}")
        dist = args.dist
    n = 1 << logn
    dev = torch.device("cuda:0")
    seed = fsgen.seed_for({"c0": 0, "c1": 1, "c2a": 2, "c2b": 2}[args.workload],
                          fsgen.valid_dists(key_bits).index(dist))
    keys = fsgen.keys_device(dist, key_bits, n, seed, device=dev)
    vals = fsgen.index_device(n, val_bytes, device=dev) if val_bytes else None
    if args.copy_probe:  # counter calibration: a plain copy of known size
        a = torch.empty(COPY_PROBE_BYTES // 4, dtype=torch.int32, device=dev).fill_(1)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    ko = torch.empty_like(keys)
    vo = torch.empty_like(vals) if vals is not None else None
    ws = fs.Workspace(dev)
    if vals is None:
        ws.get(fs.sort_keys_workspace_bytes(n, key_bits))
    else:
        ws.get(fs.sort_pairs_workspace_bytes(n, key_bits, val_bytes))
    torch.cuda.synchronize()

    def step():
        if vals is None:
            fs.sort_keys(keys, out=ko, workspace=ws)
        else:
            fs.sort_pairs(keys, vals, keys_out=ko, vals_out=vo, workspace=ws)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    print(f"[bench] warmup done ({args.warmup} steps of {desc})", file=sys.stderr, flush=True)

    L = fs.lib()
    L.fs_profile_enable(1)
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    t0.record()
    for _ in range(args.steps):
        step()
    t1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    ms_total = t0.elapsed_time(t1)
    kinds = {"histogram": 0, "plan": 1, "scatter": 2, "expand": 3, "aux": 4}
    kernels = {}
    for name, kid in kinds.items():
        c, k, ms = ctypes.c_uint64(), ctypes.c_uint64(), ctypes.c_double()
        L.fs_profile_read(kid, ctypes.byref(c), ctypes.byref(k), ctypes.byref(ms))
        kernels[name] = {"launches": c.value, "keys": k.value, "ms_total": ms.value}
    L.fs_profile_enable(0)
    if ws.error_word() != 0:
        raise SystemExit(f"device error word {ws.error_word():#x}: result invalid")

    # cheap validity check of the last result (outside the timed region)
    kk = ko.view(torch.int16).to(torch.int32) & 0xFFFF if key_bits == 16 else ko.view(
        {32: torch.int32, 64: torch.int64}[key_bits])
    if key_bits == 16:
        assert bool((kk[1:] >= kk[:-1]).all()), "output keys not sorted"
    print(f"[bench] timed {args.steps} steps in {ms_total:.1f} ms", file=sys.stderr, flush=True)

    ms_step = ms_total / args.steps
    gkeys = n * args.steps / (ms_total / 1e3) / 1e9
    active = active_digits(keys, key_bits)
    trie = False
    if key_bits == 16:
        pass_bytes = scatter_pass_bytes(key_bits, val_bytes, active) if val_bytes else []
        bpk = algorithmic_bytes_per_key(key_bits, val_bytes, active)
    else:
        # the passes the device's plan ran: one per active digit, or the
        # sparse-trie window passes followed by the fixup's read of every key
        # (and payload)
        slots, trie = plan_passes(ws)
        pass_bytes = [scatter_bytes_per_key(key_bits, val_bytes)] * len(slots)
        bpk = (key_bits // 8 + sum(pass_bytes) + (key_bits // 8 + val_bytes if trie else 0) if slots
               else algorithmic_bytes_per_key(key_bits, val_bytes, [False] * (key_bits // 8)))
    passes = len(pass_bytes)
    scatter_avg = sum(pass_bytes) / passes if passes else 0
    for name, kinfo in kernels.items():
        if kinfo["launches"]:
            kinfo["ms_avg"] = kinfo["ms_total"] / kinfo["launches"]
    dom_name = DOMINANT[args.workload]
    if key_bits == 16 and val_bytes == 0:
        dom = kernels["expand"]
        dom_bytes_per_key = 2  # the expansion writes every key once
        dom_bytes_step = n * 2
    else:
        # every scatter launch is timed, also those whose digit the device
        # found trivial (they exit at once); the bytes are those of the passes
        # that run, the time is all of it
        dom = kernels["scatter"]
        dom_bytes_per_key = scatter_avg
        dom_bytes_step = n * sum(pass_bytes)
    dom_ms_step = dom["ms_total"] / args.steps
    # with every digit trivial (all-equal keys) no pass runs: no dominant-kernel figure
    achieved = dom_bytes_step / (dom_ms_step / 1e3) / 1e9 if dom_bytes_step and dom_ms_step > 0 else None
    src_hash = kernel_source_hash()
    traffic = read_traffic(src_hash) if args.workload == "c1" and dist == "uniform" else None
    out = {
        "metric": METRIC,
        "value": round(gkeys, 3),
        "unit": "Gkeys/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {16: "u16", 32: "u32", 64: "u64"}[key_bits] + (f"+u{8 * val_bytes}" if val_bytes else ""),
        "data": "synthetic",
        "config": {"workload": desc, "n": n, "key_bits": key_bits, "val_bytes": val_bytes,
                   "distribution": dist, "seed": seed, "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "kernel": dom_name if achieved else None,
                     "achieved": round(achieved, 1) if achieved else None,
                     "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBPS, 4) if achieved else None,
                     "traffic": traffic, "bytes_per_key": dom_bytes_per_key,
                     "keys_per_launch": dom["keys"] // max(dom["launches"], 1),
                     "active_digits": [int(a) for a in active], "passes_run": passes,
                     "sparse_trie": trie},
        "hbm_frac_whole_sort": round(n * bpk / (ms_step / 1e3) / 1e9 / HBM_PEAK_GBPS, 4),
        "algorithmic_bytes_per_key": bpk,
        "kernels": {k: {kk2: (round(vv, 4) if isinstance(vv, float) else vv) for kk2, vv in v.items()}
                    for k, v in kernels.items() if v["launches"]},
        "kernel_source_sha256_16": src_hash,
        "wall_s_timed": round(wall, 3),
        # algorithmic bytes per dominant launch over the counted HBM bytes per launch
        "b_eff": (round(dom_bytes_step * args.steps / dom["launches"] / traffic, 3)
                  if traffic and dom["launches"] else None),
        "paper_context": PAPER_CONTEXT,
    }
    if args.workload == "c0":
        out["graph_replay"] = graph_replay(step, ko, args.steps)
    if not args.no_cpu_baseline:
        print("[bench] timing the CPU oracle on a sample", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(keys, vals, key_bits, val_bytes)
    print(json.dumps(out), flush=True)


def graph_replay(step, out_tensor, replays):
    """The same sort captured once into a HIP graph and replayed: the kernel
    sequence without per-launch host overhead.  The output after the replays
    is compared bit for bit with the eager result (outside the timing)."""
    import torch
    eager = out_tensor.clone()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        step()
    torch.cuda.current_stream().wait_stream(side)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        step()
    g.replay()
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record()
    for _ in range(replays):
        g.replay()
    t1.record()
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1) / replays
    same = bool(torch.equal(out_tensor, eager))
    if not same:
        raise SystemExit("graph replay output differs from the eager sort")
    n = out_tensor.numel()
    return {"ms_per_step": round(ms, 4), "gkeys_s": round(n / (ms / 1e3) / 1e9, 3), "replays": replays,
            "matches_eager": same}


if __name__ == "__main__":
    main()
