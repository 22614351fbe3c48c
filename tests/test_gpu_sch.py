"""The sphericylindrical-harmonic (SCH) appearance on the GPU
(gs4d_preprocess_sch, gs4d_preprocess_sch_bwd, gs4d_sch_from_rgb) against the
oracle (oracle.sch: FP64 colour from the conditional mean and the camera
centre; its chain rule to the coefficients and, through the viewing
direction, to the conditional mean).

* geometry of every record, tile rectangles and counts bit for bit (the
  rotor form's FP32 preprocess), colour slots within 2e-6 of the FP64 SCH
  colour (relative to the sum of its terms' magnitudes), at every degree
  0..3 and 0..2 temporal frequencies, three views at three times;
* keys, values and ranges bit for bit; the image within 1e-4;
* gradients of a random linear loss to the geometry (rows 0-16) and to all
  coefficients within 1e-3 relative of the oracle (the doubtful-decision
  bounds chained through the SCH backward, as for the rotor form);
* colour from gs4d_sch_from_rgb equals the RGB form's to FP32 rounding.
"""
import numpy as np
import pytest
import torch

import oracle
from oracle import sch as osch
from paper_2510_01119_amd import gs4d as G
from paper_2510_01119_amd import synth
from paper_2510_01119_amd.rasterizer import Rasterizer

from gpu_helpers import check_gradients, check_image, decision_bounds, need_gpu

pytestmark = pytest.mark.gpu

PERIOD = 2.0


def _views():
    vs = [synth.front_view(100, 70, 80.0, 3.0, t) for t in (0.2, 0.5)]
    vs.append(synth.make_view(synth.look_at((1.2, -0.6, -2.8), (0, 0, 0)), 80.0, 80.0, 50.0, 35.0,
                              100, 70, 0.9))
    return np.stack(vs)


def _inputs(L, N, n=3000, seed=5):
    p = synth.small_set(n, seed, log_s_xyz=(-2.5, 0.5)).astype(np.float32)
    p[17:20] = 0.0          # unused by the SCH form
    rng = np.random.default_rng(100 + 10 * L + N)
    rows = 3 * osch.n_basis(L, N)
    coef = rng.normal(0.0, 0.25, (rows, n))
    coef[0:3] = rng.uniform(0.5, 3.0, (3, n))
    coef[:, 7] = np.nan     # non-finite colour: culled in every view
    return p, coef.astype(np.float32)


def _gpu(p, coef, sch, views):
    P = torch.from_numpy(p).cuda()
    C = torch.from_numpy(coef).cuda()
    r = Rasterizer(p.shape[1], views)
    G.gs4d_preprocess_sch(P, C, sch, r.cviews, r.rec, r.rect, r.touched)
    r.bin_sort()
    r.render()
    torch.cuda.synchronize()
    return r, P, C


def _oracle_records(p, coef, views, L, N):
    """The rotor form's FP32 records with the FP64 SCH colour in slots 8-10;
    a (view, Gaussian) with a non-finite colour culled."""
    rec, rect, touched = oracle.preprocess_f32(p, views)
    mu3 = oracle.conditional_mean_all(p, views)
    col = osch.colour(coef.astype(np.float64), mu3, views, L, N, PERIOD)
    bad = ~np.all(np.isfinite(col), axis=-1)
    rec[bad] = 0.0
    rect[bad] = 0
    touched[bad] = 0
    rec64 = rec.astype(np.float64)
    vis = touched > 0
    rec64[..., 8:11] = np.where(vis[..., None], np.nan_to_num(col), 0.0)
    # magnitude scale of each colour: sum of |term|
    C = np.abs(coef.astype(np.float64)).reshape(-1, 3, p.shape[1])
    Z = np.stack([np.abs(osch.basis(L, N, PERIOD, v[18], mu3[i] - osch.camera_centres(v[None])[0]))
                  for i, v in enumerate(views)])                      # [V, n, K]
    scale = np.einsum("vgb,bcg->vgc", Z, np.nan_to_num(C))
    return rec, rect, touched, rec64, mu3, scale


@pytest.mark.parametrize("L,N", [(0, 0), (1, 1), (2, 0), (3, 2)])
def test_sch_records_and_binning(L, N):
    need_gpu()
    views = _views()
    p, coef = _inputs(L, N)
    sch = G.make_sch(L, N, PERIOD)
    r, _, _ = _gpu(p, coef, sch, views)
    rec, rect, touched, rec64, _, scale = _oracle_records(p, coef, views, L, N)
    got = r.rec.cpu().numpy()
    assert (touched > 0).sum() > 1000
    assert not touched[:, 7].any()
    assert np.array_equal(r.touched.cpu().numpy(), touched)
    assert np.array_equal(r.rect.cpu().numpy(), rect)
    geo = [0, 1, 2, 3, 4, 5, 6, 7, 11]
    assert np.array_equal(got[..., geo].view(np.uint32), rec[..., geo].view(np.uint32))
    vis = touched > 0
    err = np.abs(got[..., 8:11] - rec64[..., 8:11])
    assert np.all(err[vis] <= 2e-6 * (1.0 + scale[vis])), float(err[vis].max())
    assert np.all(got[~vis][..., 8:11] == 0.0)
    keys, vals, ranges = oracle.bin_sort(rect, touched, oracle.depth_bits(rec), views)
    P = int(r.n_pairs.item())
    assert P == len(keys)
    assert np.array_equal(r.keys[:P].cpu().numpy().view(np.uint64), keys)
    assert np.array_equal(r.vals[:P].cpu().numpy().view(np.uint32), vals)
    assert np.array_equal(r.ranges.cpu().numpy(), ranges)


@pytest.fixture(scope="module")
def sch_case():
    need_gpu()
    L, N = 3, 2
    views = _views()
    p, coef = _inputs(L, N, seed=9)
    sch = G.make_sch(L, N, PERIOD)
    r, P, C = _gpu(p, coef, sch, views)
    rec, rect, touched, rec64, mu3, _ = _oracle_records(p, coef, views, L, N)
    keys, vals, ranges = oracle.bin_sort(rect, touched, oracle.depth_bits(rec), views)
    w = synth.linear_loss_weights(r.V, r.H, r.W, seed=17)
    # the culled Gaussian's NaN coefficients reach no gradient
    c64 = np.nan_to_num(coef.astype(np.float64))
    p64 = p.astype(np.float64)

    def chain(v, g):
        dcoef, gmu = osch.backward(c64, mu3[v:v + 1], views[v:v + 1], L, N, PERIOD, g[..., 6:9],
                                   touched[v:v + 1])
        dp = oracle.preprocess_bwd(p64, views[v:v + 1], g, grad_mu3=gmu)
        return np.concatenate([dp[0:17], dcoef])

    flag, img_b, _, grad_b = decision_bounds(p, views, rec64, vals, ranges, w, chain=chain)
    return dict(L=L, N=N, views=views, p=p, coef=coef, sch=sch, r=r, P=P, C=C, rec64=rec64,
                mu3=mu3, touched=touched, vals=vals, ranges=ranges, w=w, flag=flag, img_b=img_b,
                grad_b=grad_b)


def test_sch_image(sch_case):
    c, r = sch_case, sch_case["r"]
    ref = oracle.render_fwd(c["rec64"], c["views"], c["vals"], c["ranges"], f32=True)
    check_image("sch", r.image.cpu().numpy(), ref["image"], c["flag"], c["img_b"])


def test_sch_gradients(sch_case):
    c, r = sch_case, sch_case["r"]
    L, N, views = c["L"], c["N"], c["views"]
    r.render_bwd_2d(torch.from_numpy(c["w"]).cuda())
    d = torch.full((G.N_FIELDS, r.n), 7.0, device="cuda")
    dc = torch.full_like(c["C"], 7.0)
    G.gs4d_preprocess_sch_bwd(c["P"], c["C"], c["sch"], r.touched, r.grad2d, r.cviews, d, dc)
    torch.cuda.synchronize()
    got_p, got_c = d.cpu().numpy(), dc.cpu().numpy()
    assert np.all(got_p[17:20] == 0.0)
    # a Gaussian seen by no view: every coefficient gradient written as zero
    unseen = ~np.any(c["touched"] > 0, axis=0)
    assert unseen.any() and np.all(got_c[:, unseen] == 0.0)
    grec = oracle.render_bwd(c["rec64"], views, c["vals"], c["ranges"], c["w"].astype(np.float64),
                             f32=True)
    dcoef, gmu = osch.backward(np.nan_to_num(c["coef"].astype(np.float64)), c["mu3"], views, L, N,
                               PERIOD, grec[..., 6:9], c["touched"])
    dp = oracle.preprocess_bwd(c["p"].astype(np.float64), views, grec, grad_mu3=gmu)
    ref = np.concatenate([dp[0:17], dcoef])
    got = np.concatenate([got_p[0:17], got_c])
    # the direction term reaches the mean: it is not negligible here
    dp0 = oracle.preprocess_bwd(c["p"].astype(np.float64), views, grec)
    assert np.abs(dp[0:3] - dp0[0:3]).max() > 0.05 * np.abs(dp[0:3]).max()
    check_gradients("sch", got, ref, c["grad_b"])


def test_sch_from_rgb_equals_rgb_form():
    """Coefficients from gs4d_sch_from_rgb (only the n = 0, l = 0 row set)
    give the RGB form's records (colour to FP32 rounding of rgb / Y00 * Y00)
    and image, at the largest degree and frequency count."""
    need_gpu()
    views = _views()
    p = synth.small_set(2500, 3).astype(np.float32)
    P = torch.from_numpy(p).cuda()
    sch = G.make_sch(3, 2, PERIOD)
    C = torch.full((G.gs4d_sch_rows(3, 2), p.shape[1]), 5.0, device="cuda")
    G.gs4d_sch_from_rgb(P[17:20], sch, C)
    r1 = Rasterizer(p.shape[1], views)
    r1.forward(P)
    r2 = Rasterizer(p.shape[1], views)
    G.gs4d_preprocess_sch(P, C, sch, r2.cviews, r2.rec, r2.rect, r2.touched)
    r2.bin_sort()
    r2.render()
    torch.cuda.synchronize()
    assert np.all(C[3:].cpu().numpy() == 0.0)
    assert torch.equal(r1.touched, r2.touched)
    a, b = r1.rec.cpu().numpy(), r2.rec.cpu().numpy()
    assert np.array_equal(a[..., :8], b[..., :8]) and np.array_equal(a[..., 11], b[..., 11])
    assert np.abs(a[..., 8:11] - b[..., 8:11]).max() <= 2.0 ** -22
    assert torch.equal(r1.ranges, r2.ranges)
    assert (r1.image - r2.image).abs().max().item() <= 1e-6


def test_sch_trainer_starts_as_rgb_and_trains():
    """Trainer with the SCH colour (degree 3, two frequencies), started from
    the RGB parameters: its first forward equals the RGB trainer's to FP32
    rounding; twenty steps lower the loss, move the higher coefficients off
    zero and keep everything finite."""
    need_gpu()
    from paper_2510_01119_amd.train import Trainer
    p = torch.from_numpy(synth.small_set(3000, 2)).cuda()
    views = np.stack([synth.front_view(64, 48, 60.0, 3.0, t) for t in (0.3, 0.6)])
    tgt = p.clone()
    tgt[17:20] = torch.flip(tgt[17:20], dims=[0])
    r = Rasterizer(p.shape[1], views)
    r.forward(tgt)
    targets = r.image.clone()
    rgb = Trainer(p.clone(), views, targets, budget=100)
    sch = Trainer(p.clone(), views, targets, budget=100, sch=G.make_sch(3, 2, PERIOD))
    rgb.forward_loss(0)
    a = rgb.rast.image.clone()
    sch.forward_loss(0)
    torch.cuda.synchronize()
    assert (sch.rast.image - a).abs().max().item() <= 1e-6
    l0 = sch.loss_value()
    for i in range(20):
        sch.step(i % 2)
    sch.forward_loss(0)
    torch.cuda.synchronize()
    assert sch.loss_value() < 0.9 * l0
    assert torch.isfinite(sch.coef).all() and torch.isfinite(sch.params).all()
    assert sch.coef[3:].abs().max().item() > 0.0
    assert torch.equal(sch.params[17:20], p[17:20])


def test_sch_trainer_graph_replays_match_eager():
    """The SCH trainer's step captured as HIP graphs (as the benchmark
    replays it): replays with eager work and synchronisations between them
    reproduce the eager trainer -- the first forward bit for bit, then the
    parameters and coefficients up to the reordering of the backward's float
    atomics."""
    need_gpu()
    from paper_2510_01119_amd.train import Trainer
    p = torch.from_numpy(synth.small_set(2500, 6)).cuda()
    views = np.stack([synth.front_view(64, 48, 60.0, 3.0, t) for t in (0.25, 0.5, 0.75)])
    tgt = p.clone()
    tgt[0:3] += 0.01
    r = Rasterizer(p.shape[1], views[0])
    targets = []
    for v in views:
        r.set_views(v)
        r.forward(tgt)
        targets.append(r.image.clone())
    targets = torch.cat(targets)
    sch = G.make_sch(2, 1, PERIOD)
    eager = Trainer(p.clone(), views, targets, budget=50, sch=sch)
    graph = Trainer(p.clone(), views, targets, budget=50, sch=sch)
    eager.size_pairs(margin=2.0)
    graph.size_pairs(margin=2.0)
    graph.rast._alloc_pairs(eager.rast.capacity)
    c0 = eager.coef.clone()
    frames = [0, 2, 1, 0, 2]
    graph.capture(sorted(set(frames)))
    for i, f in enumerate(frames):
        eager.step(f)
        graph.step_graph(f)
        torch.cuda.synchronize()
        _ = (eager.coef * 2).sum().item()          # eager work between replays
        if i == 0:
            assert torch.equal(eager.rast.image, graph.rast.image)
        for a, b, ref in ((eager.params, graph.params, p), (eager.coef, graph.coef, c0)):
            d = (a - b).abs().max().item()
            scale = (a - ref).abs().max().item()
            assert d <= 1e-3 * scale + 1e-7, (i, d, scale)
    assert int(graph.step_dev.item()) == len(frames)
    assert all(int(s_.item()) == len(frames) for _, _, s_ in graph.coef_groups)
    assert int(graph.overflow_seen.item()) == 0
