"""The allocation-free entry point fs_sort_keys_noalloc, called through the
C ABI, gives the same bytes as fs_sort_keys (the entry point whose kernels it
shares, with a caller-owned workspace) on the same inputs: two calls in a
row for each width, the second on a smaller input, so the second call runs
on scratch contents the first one left.  Sizes span many tiles with ragged
tails; the error word each call reports must be 0; a size whose workspace
exceeds the static array is refused before anything is launched.
"""
import numpy as np
import pytest
import torch

import fsgen
import paper_2605_10390_amd as fs

pytestmark = pytest.mark.gpu

# (key bits, clobber, first n, second n): 16-bit keys take the histogram
# path at any n; 32- and 64-bit keys take the tiled passes (clobbered or
# with the temporary copy inside the scratch array)
CASES = [(16, False, (1 << 22) + 13, 4097), (32, True, (1 << 21) + 7, 65536 + 123),
         (32, False, (1 << 20) + 5, 3 * 4096 + 17), (64, False, (1 << 20) + 3, 63),
         (64, True, 70000, 1)]


def _run_pair(bits, clobber, n, seed, dist):
    keys = fsgen.keys_device(dist, bits, n, seed)
    ref_in = keys.clone()
    ref = fs.sort_keys(ref_in, workspace=fs.Workspace(keys.device), key_type="unsigned")
    out = torch.empty_like(keys)
    err = torch.full((1,), -1, dtype=torch.int32, device=keys.device)
    fs.sort_keys_noalloc(keys, out, err_out=err, key_type="unsigned", clobber=clobber)
    torch.cuda.synchronize()
    return ref, out, int(err.item())


@pytest.mark.parametrize("bits,clobber,n1,n2", CASES)
def test_noalloc_matches_workspace_entry(gpu, bits, clobber, n1, n2):
    for i, n in enumerate((n1, n2)):
        for di, dist in enumerate(fsgen.valid_dists(bits)[:3]):
            seed = fsgen.seed_for(11, di) + 7 * n + i
            print(f"noalloc bits={bits} clobber={clobber} n={n} dist={dist} seed={seed}", flush=True)
            ref, out, err = _run_pair(bits, clobber, n, seed, dist)
            assert err == 0, (bits, n, dist, err)
            assert torch.equal(out, ref), (bits, clobber, n, dist)


def test_noalloc_empty_and_too_big(gpu):
    keys = torch.empty(0, dtype=torch.uint16, device=gpu)
    out = torch.empty_like(keys)
    err = torch.full((1,), -1, dtype=torch.int32, device=gpu)
    fs.sort_keys_noalloc(keys, out, err_out=err)
    torch.cuda.synchronize()
    assert int(err.item()) == 0
    # 2^24 32-bit keys without clobber need a 64 MiB temporary copy: refused
    big = torch.zeros(1 << 24, dtype=torch.uint32, device=gpu)
    with pytest.raises(fs.FsError) as e:
        fs.sort_keys_noalloc(big, torch.empty_like(big))
    assert e.value.status == fs.FS_ERR_WORKSPACE_TOO_SMALL
