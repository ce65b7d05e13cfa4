"""GPU parity of the batched segmented sort: every segment equals the CPU
oracle's sort of that segment alone (bit-exact), across mixed key widths,
payload widths and distributions, segment lengths on both sides of the
small-segment (in-LDS) capacity, empty and single-key segments, segments
whose every digit is trivial, and an invalid descriptor that must be
flagged without disturbing the others."""
import numpy as np
import pytest
import torch

import fsgen
import oracle
import paper_2605_10390_amd as fs

pytestmark = pytest.mark.gpu

SMALL_BYTES = 32768 - 16


def small_cap(kb, vb):
    return SMALL_BYTES // (kb + vb)


def make_segment(n, bits, vb, dist, seed, dev):
    if dist not in fsgen.valid_dists(bits):
        dist = "uniform"
    k = fsgen.keys_host(dist, bits, n, seed)
    v = fsgen.vals_host(n, vb, kind="random", seed=seed) if vb else None
    kd = torch.from_numpy(k).to(dev)
    ko = torch.empty_like(kd)
    vd = torch.from_numpy(v).to(dev) if vb else None
    vo = torch.empty_like(vd) if vb else None
    return (k, v), (kd, ko, vd, vo)


def check(host_segs, dev_segs):
    for i, ((k, v), (_, ko, _, vo)) in enumerate(zip(host_segs, dev_segs)):
        if v is None:
            assert np.array_equal(ko.cpu().numpy(), oracle.sort(k)), i
        else:
            ek, ev = oracle.sort(k, v)
            assert np.array_equal(ko.cpu().numpy(), ek), i
            assert np.array_equal(vo.cpu().numpy(), ev), i


def test_mixed_batch(gpu):
    rng = np.random.default_rng(2024)
    lengths = fsgen.lognormal_lengths(300, fsgen.seed_for(3, 9), median=600.0, sigma=2.0,
                                      cap=1 << 18)
    host, devs = [], []
    for i, n in enumerate(lengths):
        bits = (16, 32, 64)[i % 3]
        vb = (0, 4, 8)[(i // 3) % 3]
        dist = fsgen.valid_dists(bits)[rng.integers(0, len(fsgen.valid_dists(bits)))]
        h, d = make_segment(int(n), bits, vb, dist, fsgen.seed_for(5, i), gpu)
        host.append(h)
        devs.append(d)
    ws = fs.sort_segmented(devs)
    torch.cuda.synchronize()
    assert ws.error_word() == 0
    check(host, devs)


def test_capacity_edges_and_degenerate(gpu):
    host, devs = [], []
    specs = []
    for bits in (16, 32, 64):
        kb = bits // 8
        for vb in (0, 4, 8):
            c = small_cap(kb, vb)
            specs += [(0, bits, vb, "uniform"), (1, bits, vb, "uniform"), (c, bits, vb, "uniform"),
                      (c + 1, bits, vb, "uniform"), (3 * 4096 + 1, bits, vb, "uniform")]
        specs += [(50000, bits, 4, "equal" if bits == 16 else "hot90"), (70001, bits, 0, "uniform")]
    for i, (n, bits, vb, dist) in enumerate(specs):
        h, d = make_segment(n, bits, vb, dist, fsgen.seed_for(6, i), gpu)
        host.append(h)
        devs.append(d)
    # an all-equal large segment of wide keys: every digit trivial (copy path)
    n = 40000
    k = np.full(n, 0xABCDEF0123456789, dtype=np.uint64)
    kd = torch.from_numpy(k).to(gpu)
    host.append((k, None))
    devs.append((kd, torch.empty_like(kd), None, None))
    ws = fs.sort_segmented(devs)
    torch.cuda.synchronize()
    assert ws.error_word() == 0
    check(host, devs)


def test_invalid_descriptor_is_flagged(gpu):
    h0, d0 = make_segment(5000, 32, 0, "uniform", 1, gpu)
    h1, d1 = make_segment(20000, 16, 4, "zipf", 2, gpu)
    batch = fs.SegmentBatch([d0, d1])
    desc = batch.d_desc.cpu().numpy().view(fs.SEGMENT_DTYPE).copy()
    bad = np.zeros(1, dtype=fs.SEGMENT_DTYPE)
    bad[0] = (desc[0]["keys_in"], desc[0]["keys_out"], 0, 0, 10, 24, 0)  # 24-bit keys
    allx = np.concatenate([desc, bad])
    b2 = fs.SegmentBatch.from_array(allx, batch.total_keys + 10, batch.max_segment_keys,
                                    device=gpu, keep=[d0, d1])
    ws = b2.run()
    torch.cuda.synchronize()
    assert ws.error_word() & 16
    check([h0, h1], [d0, d1])


def test_segmented_repeatable(gpu):
    host, devs = [], []
    for i in range(40):
        h, d = make_segment(int(1000 + 977 * i), (16, 32)[i % 2], 0, "uniform", i, gpu)
        host.append(h)
        devs.append(d)
    batch = fs.SegmentBatch(devs)
    ws = fs.Workspace(gpu)
    batch.run(ws)
    first = [d[1].clone() for d in devs]
    batch.run(ws)
    torch.cuda.synchronize()
    for a, d in zip(first, devs):
        assert torch.equal(a.view(torch.int16 if a.dtype == torch.uint16 else torch.int32),
                           d[1].view(torch.int16 if a.dtype == torch.uint16 else torch.int32))
    check(host, devs)


def test_graph_replays_match_eager(gpu):
    """The captured launch sequence, replayed several times with eager work
    and synchronisations in between, gives the eager result every time."""
    host, devs = [], []
    for i in range(60):
        h, d = make_segment(int(300 + 4111 * (i % 7) + 37 * i), (16, 32, 64)[i % 3], (0, 4)[i % 2],
                            "uniform", 100 + i, gpu)
        host.append(h)
        devs.append(d)
    batch = fs.SegmentBatch(devs)
    ws = fs.Workspace(gpu)
    ws.get(batch.workspace_bytes())
    g = fs.CapturedSort(lambda: batch.run(ws), gpu)
    for r in range(3):
        signed = {1: torch.int8, 2: torch.int16, 4: torch.int32, 8: torch.int64}
        for d in devs:
            for t in (d[1], d[3]):
                if t is not None and t.numel():
                    t.view(signed[t.element_size()]).zero_()
        junk = torch.randn(1 << 20, device=gpu).sum()  # unrelated eager work
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert ws.error_word() == 0
        check(host, devs)
        del junk


# ---- launch tunings: every bin choice gives the same bits -------------------

NEVER = 0xFFFFFFFF
TUNINGS = [
    None,  # process-wide default
    {"small_max_keys": [NEVER] * 3, "expand16_min_keys": NEVER, "expand16_split_keys": NEVER,
     "expand16_wgs_per_cu": 1, "large_wg_max_keys": 0, "tile_items": 16, "tile_threads": 512,
     "large_wgs_per_cu": 2,
     "small_wgs_per_cu": 2},  # 8-bit digits everywhere
    {"small_max_keys": [1024, 1024, 1024], "expand16_min_keys": 1, "expand16_split_keys": 1 << 18,
     "expand16_wgs_per_cu": 2, "large_wg_max_keys": 1 << 16, "tile_items": 8, "tile_threads": 256,
     "large_wgs_per_cu": 8,
     "small_wgs_per_cu": 1},  # every 16-bit keys-only segment expanded, long ones split
    {"small_max_keys": [4096, 2048, NEVER], "expand16_min_keys": 65536, "expand16_split_keys": NEVER,
     "expand16_wgs_per_cu": 1, "large_wg_max_keys": 1 << 20, "tile_items": 8, "tile_threads": 512,
     "large_wgs_per_cu": 1,
     "small_wgs_per_cu": 4},  # long ones on one workgroup each
]


def tuned_batch(gpu):
    """16-bit keys-only segments on both sides of 65536 keys (where packed
    counters can carry), with skewed and all-equal keys whose bins pass
    65535, slices at odd element offsets (unaligned starts and ends), plus
    other widths for the other bins."""
    host, devs = [], []
    big = torch.from_numpy(fsgen.keys_host("uniform", 16, 300007, 77)).to(gpu)
    big_out = torch.full_like(big.view(torch.int16), 0xBEEF - 0x10000).view(torch.uint16)
    spec = [(1, "uniform"), (7, "uniform"), (1000, "zipf"), (4095, "uniform"), (9000, "gaussian"),
            (65535, "equal"), (65536, "zipf"), (70001, "uniform"), (200003, "zipf"),
            ((1 << 18) + 5, "uniform"), (3 * (1 << 18) + 1001, "zipf"), (1 << 20, "equal")]
    for i, (n, dist) in enumerate(spec):
        h, d = make_segment(n, 16, 0, dist, fsgen.seed_for(7, i), gpu)
        host.append(h)
        devs.append(d)
    # every key the same odd or even value: a low-half carry each 65536 keys,
    # and for the odd value carries out of the whole word
    for val, n in ((0x1234, 150001), (0x4321, 150001), (0xFFFF, 150001), (0, 150001), (0x7777, 600000)):
        k = np.full(n, val, dtype=np.uint16)
        kd = torch.from_numpy(k).to(gpu)
        host.append((k, None))
        devs.append((kd, torch.empty_like(kd), None, None))
    # two neighbouring values sharing one counter word
    k = np.where(np.arange(140000) % 3 == 0, 0x4444, 0x4445).astype(np.uint16)
    kd = torch.from_numpy(k).to(gpu)
    host.append((k, None))
    devs.append((kd, torch.empty_like(kd), None, None))
    # unaligned slices of one array (starts and ends inside 16-byte blocks)
    slices = ((1, 40000), (40003, 40013), (40021, 140021), (140029, 300000))
    for a, b in slices:
        host.append((big[a:b].cpu().numpy(), None))
        devs.append((big[a:b], big_out[a:b], None, None))
    # elements of big_out outside every slice must keep their fill
    gaps = [(0, 1), (40000, 40003), (40013, 40021), (140021, 140029), (300000, 300007)]
    for i, (n, bits, vb) in enumerate([(3000, 32, 0), (20000, 32, 4), (50000, 64, 0), (9000, 16, 4),
                                       (100000, 32, 0), (5000, 64, 8)]):
        h, d = make_segment(n, bits, vb, "uniform", fsgen.seed_for(8, i), gpu)
        host.append(h)
        devs.append(d)
    return host, devs, (big_out, gaps)


def check_gaps(guard):
    out, gaps = guard
    o = out.cpu().numpy()
    for a, b in gaps:
        assert (o[a:b] == 0xBEEF).all(), (a, b)


@pytest.mark.parametrize("ti", range(len(TUNINGS)))
def test_every_tuning_is_bit_exact(gpu, ti):
    host, devs, guard = tuned_batch(gpu)
    t = fs.SegTuning.from_dict(TUNINGS[ti]) if TUNINGS[ti] else None
    ws = fs.sort_segmented(devs, tuning=t)
    torch.cuda.synchronize()
    assert ws.error_word() == 0
    check(host, devs)
    check_gaps(guard)


def test_autotuner_picks_a_valid_tuning(gpu):
    from paper_2605_10390_amd import autotune
    host, devs, guard = tuned_batch(gpu)
    batch = fs.SegmentBatch(devs)
    ws = fs.Workspace(gpu)
    best, report = autotune.tune_batch(batch, ws, reps=1, sweeps=1)
    assert report["best_ms"] <= report["start_ms"]
    signed = {2: torch.int16, 4: torch.int32, 8: torch.int64}
    for d in devs:
        for t in (d[1], d[3]):
            if t is not None and t.numel():
                t.view(signed[t.element_size()]).zero_()
    batch.run(ws, tuning=best)
    torch.cuda.synchronize()
    assert ws.error_word() == 0
    check(host, devs)


def test_large_bin_histograms_start_from_zero(gpu):
    """Regression: the large-bin digit histograms must be cleared before any
    wave counts into them.  Many 16-bit keys-only segments through the large
    bin with eight workgroups per CU (short per-workgroup stretches, where a
    missing barrier after the clear lost counts), repeated."""
    host, devs = [], []
    for i in range(24):
        h, d = make_segment(150000 + 4099 * i, 16, 0, ("uniform", "zipf")[i % 2], fsgen.seed_for(9, i), gpu)
        host.append(h)
        devs.append(d)
    t = fs.SegTuning.from_dict({"small_max_keys": [NEVER] * 3, "expand16_min_keys": NEVER,
                                "expand16_split_keys": NEVER, "expand16_wgs_per_cu": 1,
                                "large_wg_max_keys": 0, "tile_items": 8, "tile_threads": 256,
                                "large_wgs_per_cu": 8, "small_wgs_per_cu": 2})
    batch = fs.SegmentBatch(devs)
    ws = fs.Workspace(gpu)
    for _ in range(6):
        batch.run(ws, tuning=t)
        torch.cuda.synchronize()
        assert ws.error_word() == 0
        check(host, devs)


def test_wave_bin_tiny_segments(gpu):
    """Segments of 1..64 keys (the wave bin) of every width and payload,
    with repeated keys, in every key order, next to longer segments."""
    rng = np.random.default_rng(64)
    specs = []
    for i in range(300):
        bits = (16, 32, 64)[i % 3]
        vb = (0, 4, 8)[(i // 3) % 3]
        n = int(rng.integers(1, 65)) if i % 10 else 64
        specs.append((bits, vb, n))
    specs += [(32, 4, 65), (16, 0, 5000)]
    for key_type, desc in (("unsigned", False), ("signed", True), ("float", False)):
        segs, want = [], []
        for bits, vb, n in specs:
            k = rng.integers(0, 1 << 63, n, dtype=np.uint64).astype({16: np.uint16, 32: np.uint32, 64: np.uint64}[bits])
            k[: n // 3] = k[n // 3: 2 * (n // 3)]
            v = rng.integers(0, 1 << 32, n, dtype=np.uint64).astype(np.uint32 if vb == 4 else np.uint64) if vb else None
            ki = torch.from_numpy(k).cuda()
            vi = torch.from_numpy(v).cuda() if vb else None
            segs.append((ki, torch.empty_like(ki), vi, torch.empty_like(vi) if vb else None))
            want.append(oracle.sort_ordered(k, v, key_type=key_type, descending=desc))
        ws = fs.sort_segmented(segs, key_type=key_type, descending=desc)
        torch.cuda.synchronize()
        assert ws.error_word() == 0
        for (bits, vb, n), (_, ko, _, vo), w in zip(specs, segs, want):
            if vo is None:
                assert np.array_equal(ko.cpu().numpy(), w), (key_type, bits, vb, n)
            else:
                assert np.array_equal(ko.cpu().numpy(), w[0]), (key_type, bits, vb, n)
                assert np.array_equal(vo.cpu().numpy(), w[1]), (key_type, bits, vb, n)
