"""The crop evaluation used by the differentiation-at-scale checks, against
the plain oracle pipeline: restricting to the Gaussians that meet the crop
leaves every crop pixel unchanged, and the incremental re-insertion of a
moved Gaussian renders the same pixels, bit for bit, as a full re-sort."""
import numpy as np

import oracle
from paper_2510_01119_amd import synth

from crop_oracle import CropFD, densest_crop


def _setup():
    p = synth.clustered_set(20_000, seed=4)
    view = synth.front_view(256, 160, 200.0, 3.0, 0.5)
    rec, rect, touched = oracle.preprocess_f32(p, view)
    crop, pairs = densest_crop(view, rect, touched, size=4)
    return p, view, crop, rect, touched, pairs


def _crop_image(q, view, crop):
    rec, rect, touched = oracle.preprocess_f64(q, view)
    _, vals, ranges = oracle.bin_sort(rect, touched, oracle.depth_bits(rec), view)
    return oracle.render_fwd(rec, view, vals, crop.restrict(ranges), f32=False)["image"][0]


def test_subset_restriction_exact():
    p, view, crop, rect, touched, pairs = _setup()
    assert pairs > 0
    sub = np.nonzero(crop.meets(rect, touched))[0]
    assert 0 < len(sub) < p.shape[1]
    full = _crop_image(p.astype(np.float64), view, crop)
    part = _crop_image(p[:, sub].astype(np.float64), view, crop)
    m = crop.pixel_mask()
    assert np.array_equal(full[:, m], part[:, m])
    assert np.abs(full[:, m]).max() > 0


def test_incremental_move_matches_full_sort():
    p, view, crop, rect, touched, _ = _setup()
    sub = np.nonzero(crop.meets(rect, touched))[0]
    ps = p[:, sub].astype(np.float64)
    w = synth.linear_loss_weights(1, 160, 256, 3)
    fd = CropFD(ps, crop, w)
    rng = np.random.default_rng(2)
    for _ in range(6):
        g, k = int(rng.integers(0, len(sub))), int(rng.integers(0, 20))
        for step in (0.05, -0.05):        # large enough to reorder depths and tiles
            col = ps[:, g].copy()
            col[k] += step
            moved = fd.moved(g, col)
            tiles = fd._tiles_of(fd.rect[0, g], fd.touched[0, g]) | fd._tiles_of(moved[1], moved[2])
            if not tiles:
                continue
            _, _, pix = fd._render(g, *moved, tiles)
            q = ps.copy()
            q[k, g] += step
            ref = _crop_image(q, view, crop)
            m = np.zeros(crop.tx * crop.ty, bool)
            m[list(tiles)] = True
            pm = np.repeat(np.repeat(m.reshape(crop.ty, crop.tx), 16, 0), 16, 1)[:crop.H, :crop.W]
            assert np.array_equal(pix, ref[:, pm]), (g, k, step)
