"""Autotuner of the batched segmented sort (fs_sort_segmented_tuned).

The paper sizes its batches by measurement rather than by formula
(Section III-C); here the same is done for the launch of a segmented sort.
Segments are binned on the device by width and length, and a tuning
(fs_seg_tuning) fixes, per bin:
  - the digit width: 16-bit keys without payload from `expand16_min_keys`
    on use one 16-bit digit (compressed histogram + expansion), the rest
    8-bit digits;
  - how many workgroups sort one segment: one (the LDS bin, up to
    `small_max_keys[w]` keys, or the 16-bit-digit bin) or many (the large
    bin, in tiles);
  - the tile size of the large bin (`tile_items` x `tile_threads`) and the workgroups per
    compute unit of the LDS and large bins.
Every tuning gives bit-identical output, so the tuner only times.

The search is a coordinate descent: starting from a tuning, each field in
turn is set to each of its candidate values with the others held, and the
fastest value is kept when it beats the current time by more than a noise
margin; sweeps repeat until one changes nothing (or a sweep limit).
`coordinate_search` is pure host logic over a `measure(tuning_dict) -> ms`
callback; `tune_batch` measures a device-resident SegmentBatch with HIP
events.
"""
import itertools
import json
import statistics

NEVER = 0xFFFFFFFF

# candidate values of every tuning field; "small_max_keys" is searched per key width
CANDIDATES = {
    "expand16_min_keys": [NEVER, 1024, 2048, 4096, 8192, 16384, 32768, 65536],
    "expand16_split_keys": [1 << 18, 1 << 19, 1 << 20, 1 << 21, NEVER],
    "expand16_wgs_per_cu": [1, 2],
    "small_max_keys.0": [1024, 2048, 4096, 8192, NEVER],
    "small_max_keys.1": [1024, 2048, 4096, NEVER],
    "small_max_keys.2": [1024, 2048, NEVER],
    "large_wg_max_keys": [0, 1 << 15, 1 << 16, 1 << 17, 1 << 18, 1 << 19, 1 << 20, 1 << 21],
    "tile_items": [8, 16],
    "tile_threads": [256, 512],
    "large_wgs_per_cu": [1, 2, 3, 4, 6, 8],
    "small_wgs_per_cu": [1, 2],
}
# search order; a tuple is a group of coupled fields searched over their
# product (the tile size decides how many workgroups fit on a CU)
ORDER = ["expand16_min_keys", "expand16_split_keys", "expand16_wgs_per_cu", "small_max_keys.0",
         "small_max_keys.1", "small_max_keys.2", "large_wg_max_keys",
         ("tile_items", "tile_threads", "large_wgs_per_cu"), "small_wgs_per_cu"]


def get_field(t, name):
    if name.startswith("small_max_keys."):
        return t["small_max_keys"][int(name.split(".")[1])]
    return t[name]


def with_field(t, name, value):
    u = {k: (list(v) if isinstance(v, list) else v) for k, v in t.items()}
    if name.startswith("small_max_keys."):
        u["small_max_keys"][int(name.split(".")[1])] = value
    else:
        u[name] = value
    return u


def key_of(t):
    return json.dumps(t, sort_keys=True)


def coordinate_search(measure, start, candidates=None, order=None, sweeps=3, margin=0.01):
    """Coordinate descent over the tuning fields.

    measure(t) -> milliseconds for tuning dict t (called once per distinct
    tuning; results are cached).  A candidate replaces the current value only
    when it is faster by more than `margin` (relative), so measurement noise
    does not make the search wander.  Returns (best tuning, best ms, history)
    where history lists (tuning, ms) in measurement order."""
    candidates = candidates or CANDIDATES
    order = order or ORDER
    cache, history = {}, []

    def timed(t):
        k = key_of(t)
        if k not in cache:
            cache[k] = float(measure(t))
            history.append((t, cache[k]))
        return cache[k]

    best = {k: (list(v) if isinstance(v, list) else v) for k, v in start.items()}
    best_ms = timed(best)
    for _ in range(sweeps):
        changed = False
        for entry in order:
            names = entry if isinstance(entry, tuple) else (entry,)
            trials = []
            for values in itertools.product(*(candidates[nm] for nm in names)):
                t = best
                for nm, v in zip(names, values):
                    t = with_field(t, nm, v)
                moved = sum(get_field(t, nm) != get_field(best, nm) for nm in names)
                trials.append((timed(t), moved, t))
            fastest = min(ms for ms, _, _ in trials)
            if fastest < best_ms * (1.0 - margin):
                # among the trials within the margin of the fastest, the one
                # that changes the fewest fields
                ms, _, t = min((tr for tr in trials if tr[0] <= fastest * (1.0 + margin)),
                               key=lambda tr: (tr[1], tr[0]))
                best, best_ms, changed = t, ms, True
        if not changed:
            break
    return best, best_ms, history


def tune_batch(batch, workspace, reps=3, sweeps=2, margin=0.01, start=None, stream=None, log=None):
    """Tune the launch of `batch` (a SegmentBatch) on its own data.

    Every candidate is run once untimed, then `reps` times between HIP
    events on the current stream; its time is the median.  Returns
    (SegTuning, report dict)."""
    import torch
    import paper_2605_10390_amd as fs

    dev = batch.d_desc.device
    s = stream if stream is not None else torch.cuda.current_stream(dev)
    workspace.get(batch.workspace_bytes())

    def measure(t):
        tt = fs.SegTuning.from_dict(t)
        batch.run(workspace, stream=s, tuning=tt)
        times = []
        for _ in range(reps):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(s)
            batch.run(workspace, stream=s, tuning=tt)
            b.record(s)
            b.synchronize()
            times.append(a.elapsed_time(b))
        if workspace.error_word() != 0:
            raise RuntimeError(f"device error word {workspace.error_word():#x} under tuning {t}")
        ms = statistics.median(times)
        if log:
            log(f"[autotune] {ms:8.3f} ms  {t}")
        return ms

    start = start or fs.get_tuning().as_dict()
    best, best_ms, history = coordinate_search(measure, start, sweeps=sweeps, margin=margin)
    report = {"start": start, "start_ms": history[0][1], "best": best, "best_ms": best_ms,
              "measured": len(history)}
    return fs.SegTuning.from_dict(best), report


def save(path, tuning, report=None):
    with open(path, "w") as f:
        json.dump({"tuning": tuning.as_dict(), "report": report}, f, indent=1, sort_keys=True)


def load(path):
    import paper_2605_10390_amd as fs
    with open(path) as f:
        return fs.SegTuning.from_dict(json.load(f)["tuning"])
