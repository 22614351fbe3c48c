"""gs4d_bin_sort_noalloc (no workspace argument: the library's own device
scratch) against gs4d_bin_sort through the C ABI: pair count, overflow
flag, sort keys, values and tile ranges bit-identical, on two calls in a
row, the second with a smaller input (the scratch then holds the first
call's contents); the regular call's workspace is filled with garbage
first, so neither path relies on cleared scratch.  A call whose workspace
would exceed the scratch is refused on the host."""
import numpy as np
import pytest
import torch

from paper_2510_01119_amd import gs4d as G
from paper_2510_01119_amd import synth

from gpu_helpers import need_gpu

pytestmark = pytest.mark.gpu


def _inputs(n, seed, W, H):
    p = synth.small_set(n, seed, log_s_xyz=(-3.2, 0.5))
    vs = np.stack([synth.front_view(W, H, 0.8 * W, 3.0, t) for t in (0.35, 0.6)])
    P = torch.from_numpy(p).cuda()
    V = len(vs)
    rec = torch.zeros((V, n, G.REC_FLOATS), device="cuda")
    rect = torch.zeros((V, n, 4), dtype=torch.int32, device="cuda")
    touched = torch.zeros((V, n), dtype=torch.int32, device="cuda")
    cv = G.make_views(vs)
    G.gs4d_preprocess(P, cv, rec, rect, touched)
    return rec, rect, touched, cv, n


def _run(inputs, capacity, noalloc):
    rec, rect, touched, cv, n = inputs
    V = len(cv)
    tiles = V * ((cv[0].width + 15) // 16) * ((cv[0].height + 15) // 16)
    keys = torch.full((capacity,), -1, dtype=torch.int64, device="cuda")
    vals = torch.full((capacity,), -1, dtype=torch.int32, device="cuda")
    ranges = torch.full((tiles, 2), -7, dtype=torch.int32, device="cuda")
    n_pairs = torch.zeros(1, dtype=torch.int64, device="cuda")
    overflow = torch.full((1,), 5, dtype=torch.int32, device="cuda")
    if noalloc:
        G.gs4d_bin_sort_noalloc(rec, rect, touched, n, cv, capacity, keys, vals, ranges, n_pairs,
                                overflow)
    else:
        ws = torch.full((G.gs4d_bin_sort_workspace_size(n, V, capacity),), 0xAB, dtype=torch.uint8,
                        device="cuda")
        G.gs4d_bin_sort(rec, rect, touched, n, cv, capacity, keys, vals, ranges, n_pairs, overflow,
                        ws)
    torch.cuda.synchronize()
    P = int(n_pairs.item())
    return (P, int(overflow.item()), keys[:min(P, capacity)].cpu().numpy(),
            vals[:min(P, capacity)].cpu().numpy(), ranges.cpu().numpy())


def test_noalloc_equals_bin_sort():
    need_gpu()
    # two calls in a row, the second smaller; then one over its pair capacity
    for n, seed, W, H, cap in ((20000, 1, 320, 180, 600_000), (3000, 2, 160, 96, 60_000),
                               (3000, 2, 160, 96, 500)):
        inputs = _inputs(n, seed, W, H)
        ref = _run(inputs, cap, noalloc=False)
        got = _run(inputs, cap, noalloc=True)
        assert ref[0] == got[0] and ref[1] == got[1], (n, ref[:2], got[:2])
        if ref[1] == 0:
            assert ref[0] > 1000
            assert np.array_equal(ref[2], got[2]) and np.array_equal(ref[3], got[3])
            assert np.array_equal(ref[4], got[4])
        else:
            assert ref[0] > cap


def test_noalloc_refuses_oversized_call():
    need_gpu()
    inputs = _inputs(1000, 3, 64, 64)
    rec, rect, touched, cv, n = inputs
    big = 1 << 30
    assert G.gs4d_bin_sort_workspace_size(n, len(cv), big) > (64 << 20)
    dummy = torch.zeros(1, dtype=torch.int64, device="cuda")
    with pytest.raises(G.GS4DError, match="scratch"):
        G.gs4d_bin_sort_noalloc(rec, rect, touched, n, cv, big, dummy, dummy, dummy, dummy, dummy)
