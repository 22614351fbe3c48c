"""The isotropic, motion-aware parameterisation on the GPU (gs4d_preprocess_iso
and gs4d_preprocess_iso_bwd) against the oracle.

* records, tile rectangles and counts bit for bit (FP32, same operation
  order), and the binning of those records bit for bit, on a moving set
  seen at three times, including non-finite and zero-velocity Gaussians;
* the gradients of a random linear loss through the render backward and the
  isotropic preprocess backward against the oracle's FP64 chain rule, to
  1e-3 relative (Gaussians seen at a pixel next to a threshold exempted, as
  for the rotor form).
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2510_01119_amd import gs4d as G
from paper_2510_01119_amd import synth
from paper_2510_01119_amd.rasterizer import Rasterizer

from gpu_helpers import check_gradients, decision_bounds, need_gpu

pytestmark = pytest.mark.gpu


def _iso_params(n, seed):
    rng = np.random.default_rng(seed)
    p = np.zeros((G.ISO_FIELDS, n))
    p[0:3] = rng.uniform(-1.0, 1.0, (3, n))
    p[3] = rng.uniform(0.0, 1.0, n)
    p[4] = rng.normal(-3.0, 0.5, n)
    p[5] = rng.normal(-1.5, 0.5, n)
    p[6:9] = rng.normal(0.0, 0.5, (3, n))
    p[6:9, : n // 10] = 0.0
    p[9] = rng.normal(0.0, 1.0, n)
    p[10:13] = rng.uniform(0.0, 1.0, (3, n))
    p[0, n // 10] = np.nan
    p[5, n // 10 + 1] = np.inf
    return p.astype(np.float32)


def _gpu_iso(p, views):
    P = torch.from_numpy(p).cuda()
    r = Rasterizer(p.shape[1], views)
    G.gs4d_preprocess_iso(P, r.cviews, r.rec, r.rect, r.touched)
    r.bin_sort()
    r.render()
    torch.cuda.synchronize()
    return r, P


@pytest.fixture(scope="module")
def iso_case():
    need_gpu()
    p = _iso_params(4000, 7)
    views = np.stack([synth.front_view(100, 70, 80.0, 3.0, t) for t in (0.2, 0.5, 0.9)])
    r, P = _gpu_iso(p, views)
    rec, rect, touched = oracle.preprocess_iso_f32(p, views)
    keys, vals, ranges = oracle.bin_sort(rect, touched, oracle.depth_bits(rec), views)
    return dict(p=p, views=views, r=r, P=P, rec=rec, rect=rect, touched=touched, keys=keys,
                vals=vals, ranges=ranges)


def test_iso_preprocess_and_binning_bitexact(iso_case):
    c, r = iso_case, iso_case["r"]
    assert (c["touched"] > 0).sum() > 1000
    assert np.array_equal(r.touched.cpu().numpy(), c["touched"])
    assert np.array_equal(r.rect.cpu().numpy(), c["rect"])
    assert np.array_equal(r.rec.cpu().numpy().view(np.uint32), c["rec"].view(np.uint32))
    P = int(r.n_pairs.item())
    assert P == len(c["keys"])
    assert np.array_equal(r.keys[:P].cpu().numpy().view(np.uint64), c["keys"])
    assert np.array_equal(r.vals[:P].cpu().numpy().view(np.uint32), c["vals"])
    assert np.array_equal(r.ranges.cpu().numpy(), c["ranges"])


def test_iso_gradients(iso_case):
    c, r = iso_case, iso_case["r"]
    V, H, W = r.V, r.H, r.W
    w = synth.linear_loss_weights(V, H, W, seed=13)
    r.render_bwd_2d(torch.from_numpy(w).cuda())
    d = torch.zeros((G.ISO_FIELDS, r.n), device="cuda")
    G.gs4d_preprocess_iso_bwd(c["P"], r.touched, r.grad2d, r.cviews, d)
    torch.cuda.synchronize()
    got = d.cpu().numpy()
    rec64 = c["rec"].astype(np.float64)
    grec = oracle.render_bwd(rec64, c["views"], c["vals"], c["ranges"], w.astype(np.float64),
                             f32=True)
    ref = oracle.preprocess_iso_bwd(c["p"].astype(np.float64), c["views"], grec)
    _, _, _, gb = decision_bounds(c["p"], c["views"], rec64, c["vals"], c["ranges"], w, iso=True)
    check_gradients("iso", got, ref, gb)


def test_iso_trainer_starts_as_rotor_and_trains():
    """Trainer on isotropic parameters converted from an identity-rotor,
    tied-scale set: the first forward equals the rotor form's bit for bit
    (the same model at zero velocity); twenty steps lower the loss and keep
    the parameters finite."""
    need_gpu()
    from paper_2510_01119_amd.train import Trainer, to_iso
    rng = np.random.default_rng(3)
    n = 3000
    p = np.zeros((G.N_FIELDS, n), np.float32)
    p[0:3] = rng.uniform(-1, 1, (3, n))
    p[3] = rng.uniform(0, 1, n)
    p[4:7] = rng.normal(-3.0, 0.3, n)
    p[7] = rng.normal(-1.0, 0.3, n)
    p[8] = 1.0
    p[12] = 1.0
    p[16] = rng.normal(0, 1, n)
    p[17:20] = rng.uniform(0, 1, (3, n))
    views = np.stack([synth.front_view(64, 48, 60.0, 3.0, t) for t in (0.3, 0.6)])
    P = torch.from_numpy(p).cuda()
    tgt_p = P.clone()
    tgt_p[0:3] += 0.02
    r = Rasterizer(n, views)
    r.forward(tgt_p)
    targets = r.image.clone()
    rot = Trainer(P.clone(), views, targets, budget=100)
    iso = Trainer(to_iso(P), views, targets, budget=100)
    assert iso.params.shape == (G.ISO_FIELDS, n) and iso.cfg.rows == G.ISO_FIELDS
    rot.forward_loss(0)
    iso.forward_loss(0)
    torch.cuda.synchronize()
    assert torch.equal(rot.rast.image, iso.rast.image)
    first = iso.loss_value()
    for k in range(20):
        iso.step(k % 2)
    iso.forward_loss(0)
    torch.cuda.synchronize()
    assert iso.loss_value() < first
    assert torch.isfinite(iso.params).all()
    assert float(iso.params[6:9].abs().max()) > 0.0   # the velocity is trained
