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
