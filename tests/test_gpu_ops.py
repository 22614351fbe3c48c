"""GPU parity of the optimisation-loop kernels (Adam, L1, SSIM, squared
error) and of the grid prune against the oracle, through the C ABI."""
import numpy as np
import pytest
import torch

from oracle import adam as oadam
from oracle import losses as olosses
import oracle
from paper_2510_01119_amd import gs4d as G

from gpu_helpers import need_gpu

pytestmark = pytest.mark.gpu


def _dev(a, offset):
    """a on the device, starting `offset` floats into its allocation (offset 1
    leaves the data 4-byte but not 16-byte aligned)."""
    t = torch.zeros(a.size + offset, dtype=torch.float32, device="cuda")
    v = t[offset:].view(a.shape)
    v.copy_(torch.from_numpy(np.ascontiguousarray(a)))
    return v


@pytest.mark.parametrize("n,rows,frozen,offset", [
    (5000, 20, None, 0),
    # row boundaries inside groups of four elements, a ragged tail of
    # rows * n % 4 = 1 elements, and a frozen row (rate 0)
    (5001, 13, 3, 0),
    # arrays not 16-byte aligned (the one-element-per-thread kernel)
    (5001, 13, 3, 1),
])
def test_adam_matches_oracle(n, rows, frozen, offset):
    """Five Adam steps with a decaying per-row learning rate.  Parameters
    start at 0 so that FP32 resolves the ~lr-sized displacements.  A row
    whose rate is 0 is left untouched, moments included."""
    need_gpu()
    rng = np.random.default_rng(0)
    p = np.zeros((rows, n), np.float32)
    cfg = G.gs4d_adam_cfg()
    lr0 = np.array([1e-5] * 4 + [5e-3] * 4 + [1e-3] * 8 + [5e-2] + [2.5e-3] * 3, np.float32)[:rows]
    if frozen is not None:
        lr0[frozen] = 0.0
    lr1 = lr0 * 0.01
    for k in range(rows):
        cfg.lr0[k] = float(lr0[k])
        cfg.lr1[k] = float(lr1[k])
    cfg.budget, cfg.rows, cfg.beta1, cfg.beta2, cfg.eps = 100, rows, 0.9, 0.999, 1e-15
    P = _dev(p, offset)
    M = _dev(np.zeros_like(p), offset)
    V = _dev(np.zeros_like(p), offset)
    step = torch.zeros(1, dtype=torch.int32, device="cuda")
    rp, rm, rv = p.astype(np.float64), np.zeros((rows, n)), np.zeros((rows, n))
    live = [k for k in range(rows) if k != frozen]
    for s in range(1, 6):
        g = rng.normal(0, 1, (rows, n)).astype(np.float32)
        G.gs4d_adam_step(P, _dev(g, offset), M, V, cfg, step)
        lrs = [oadam.lr_schedule(s, float(lr0[k]), float(lr1[k]), 100) if k != frozen else 0.0
               for k in range(rows)]
        rp, rm, rv = oadam.adam_step(rp, g, rm, rv, s, lrs, eps=1e-15)
    torch.cuda.synchronize()
    assert int(step.item()) == 5
    gm, gv = M.cpu().numpy(), V.cpu().numpy()
    assert np.allclose(gm[live], rm[live], rtol=1e-5, atol=1e-7)
    # beta2 = 0.999 is not representable in FP32: 1 - fl32(0.999) differs
    # from 0.001 by 1.3e-5 relative, which the second moment inherits
    assert np.allclose(gv[live], rv[live], rtol=5e-5, atol=1e-9)
    got = P.cpu().numpy().astype(np.float64)
    for k in live:
        assert np.allclose(got[k], rp[k], rtol=1e-4, atol=1e-5 * lr0[k])
    if frozen is not None:
        assert not got[frozen].any() and not gm[frozen].any() and not gv[frozen].any()


@pytest.mark.parametrize("shape", [(1, 3, 64, 64), (2, 3, 37, 50)])
def test_l1_ssim_sse_match_oracle(shape):
    need_gpu()
    rng = np.random.default_rng(1)
    x = rng.uniform(0, 1, shape).astype(np.float32)
    y = np.clip(x + rng.normal(0, 0.1, shape), 0, 1).astype(np.float32)
    X, Y = torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda()
    loss = torch.zeros(1, device="cuda")
    dl = torch.zeros_like(X)
    G.gs4d_loss_l1(X, Y, 0.8, loss, dl)
    ssim = torch.zeros(1, device="cuda")
    ds = torch.zeros_like(X)
    ws = torch.zeros(G.gs4d_ssim_workspace_size(*shape), dtype=torch.uint8, device="cuda")
    G.gs4d_ssim(X, Y, 1.0, ssim, ds, ws)
    sse = torch.zeros(1, dtype=torch.float64, device="cuda")
    G.gs4d_sse(X, Y, sse)
    torch.cuda.synchronize()
    l1v, l1g = olosses.l1(x, y)
    assert np.isclose(loss.item(), 0.8 * l1v, rtol=1e-5)
    assert np.allclose(dl.cpu().numpy(), 0.8 * l1g, rtol=1e-6, atol=1e-12)
    sv, sg = 0.0, np.zeros(shape)
    for b in range(shape[0]):
        v_, g_ = olosses.ssim(x[b], y[b])
        sv += v_ / shape[0]
        sg[b] = g_ / shape[0]
    assert np.isclose(ssim.item(), sv, rtol=1e-4)
    g_gpu = ds.cpu().numpy()
    assert np.abs(g_gpu - sg).max() <= 1e-3 * np.abs(sg).max()
    assert np.isclose(sse.item(), ((x.astype(np.float64) - y) ** 2).sum(), rtol=1e-9)


def _points(m, seed):
    rng = np.random.default_rng(seed)
    xyz = rng.normal(0, 0.3, (3, m)).astype(np.float32)
    attr = rng.uniform(0, 1, (5, m)).astype(np.float32)
    cls = (rng.uniform(0, 1, m) < 0.3).astype(np.uint8)
    return xyz, attr, cls


# 9M points: the point scans span more than 2048 blocks of 4096 and take
# the three-kernel scan (block sums scanned by one block); smaller ones fuse it
@pytest.mark.parametrize("m,vs,vd,min_count", [(20000, 0.02, 0.02, 1), (50000, 0.05, 0.01, 3),
                                               (30000, 0.03, 0.0, 1), (7, 0.5, 0.5, 1),
                                               (9_000_000, 0.01, 0.005, 1)])
def test_grid_prune_matches_oracle(m, vs, vd, min_count):
    need_gpu()
    xyz, attr, cls = _points(m, m)
    ref = oracle.grid_prune(xyz, attr, cls, vs, vd, min_count)
    cap = m
    dev = "cuda"
    X, A, C = (torch.from_numpy(a).to(dev) for a in (xyz, attr, cls))
    ox = torch.zeros((3, cap), device=dev)
    oa = torch.zeros((5, cap), device=dev)
    oc = torch.zeros(cap, dtype=torch.int32, device=dev)
    ok = torch.zeros(cap, dtype=torch.int64, device=dev)
    nout = torch.zeros(1, dtype=torch.int64, device=dev)
    status = torch.zeros(1, dtype=torch.int32, device=dev)
    ws = torch.zeros(G.gs4d_grid_prune_workspace_size(m, 5), dtype=torch.uint8, device=dev)
    G.gs4d_grid_prune(X, A, C, vs, vd, min_count, cap, ox, oa, oc, ok, nout, status, ws)
    torch.cuda.synchronize()
    assert status.item() == 0
    k = int(nout.item())
    assert k == len(ref["count"])
    assert np.array_equal(ok[:k].cpu().numpy().view(np.uint64), ref["key"])
    assert np.array_equal(oc[:k].cpu().numpy(), ref["count"])
    assert np.allclose(ox[:, :k].cpu().numpy(), ref["xyz"], rtol=1e-6, atol=1e-7)
    assert np.allclose(oa[:, :k].cpu().numpy(), ref["attr"], rtol=1e-6, atol=1e-7)


def test_grid_prune_capacity_and_range_flags():
    need_gpu()
    xyz, attr, cls = _points(5000, 3)
    dev = "cuda"
    X = torch.from_numpy(xyz).to(dev)
    cap = 10
    outs = [torch.zeros((3, cap), device=dev), torch.zeros(cap, dtype=torch.int32, device=dev),
            torch.zeros(cap, dtype=torch.int64, device=dev)]
    nout = torch.zeros(1, dtype=torch.int64, device=dev)
    status = torch.zeros(1, dtype=torch.int32, device=dev)
    ws = torch.zeros(G.gs4d_grid_prune_workspace_size(5000, 0), dtype=torch.uint8, device=dev)
    G.gs4d_grid_prune(X, None, None, 0.01, 0.01, 1, cap, outs[0], None, outs[1], outs[2], nout,
                      status, ws)
    torch.cuda.synchronize()
    assert status.item() == 1 and nout.item() > cap
    # voxel index outside [-2^19, 2^19)
    G.gs4d_grid_prune(X, None, None, 1e-7, 1e-7, 1, cap, outs[0], None, outs[1], outs[2], nout,
                      status, ws)
    torch.cuda.synchronize()
    assert status.item() == 2


@pytest.mark.parametrize("shape", [(1, 3, 64, 64), (1, 3, 37, 50)])
def test_photometric_loss_matches_oracle(shape):
    """loss = L1 + 0.2 (1 - SSIM) and its gradient in one call."""
    need_gpu()
    rng = np.random.default_rng(2)
    x = rng.uniform(0, 1, shape).astype(np.float32)
    y = np.clip(x + rng.normal(0, 0.1, shape), 0, 1).astype(np.float32)
    X, Y = torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda()
    loss = torch.full((1,), 123.0, device="cuda")
    d = torch.full_like(X, 7.0)           # overwritten, not accumulated
    ws = torch.zeros(G.gs4d_photometric_loss_workspace_size(*shape), dtype=torch.uint8,
                     device="cuda")
    for _ in range(2):                     # a second call gives the same result
        G.gs4d_photometric_loss(X, Y, 1.0, 0.2, loss, d, ws)
        torch.cuda.synchronize()
        lv, g = olosses.scene_loss(x[0], y[0])
        assert np.isclose(loss.item(), lv, rtol=1e-5)
        gg = d.cpu().numpy()[0]
        assert np.abs(gg - g).max() <= 1e-3 * np.abs(g).max()
