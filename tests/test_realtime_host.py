"""Host side of the forward-only path: a rescaled camera maps every point to
the pixel position scaled by the image-size ratio (pinhole projection
u = fx x/z + cx, v = fy y/z + cy in camera coordinates)."""
import numpy as np

from paper_2510_01119_amd import synth
from paper_2510_01119_amd.realtime import DISPLAY_SIZES, rescale_view


def _project(view, pts):
    Rt = view[0:12].reshape(3, 4)
    cam = pts @ Rt[:, :3].T + Rt[:, 3]
    fx, fy, cx, cy = view[12:16]
    return np.stack([fx * cam[:, 0] / cam[:, 2] + cx, fy * cam[:, 1] / cam[:, 2] + cy], axis=1)


def test_rescale_view_scales_pixel_positions():
    rng = np.random.default_rng(0)
    base = synth.make_view(synth.look_at((0.3, -0.2, -3.0), (0.0, 0.0, 0.0)), 800.0, 790.0,
                           481.0, 268.0, 960, 540, 0.4)
    pts = rng.uniform(-1, 1, (50, 3))
    uv = _project(base, pts)
    for W, H in DISPLAY_SIZES:
        v = rescale_view(base, W, H)
        assert int(v[16]) == W and int(v[17]) == H
        assert np.array_equal(v[0:12], base[0:12]) and np.array_equal(v[18:], base[18:])
        got = _project(v, pts)
        assert np.allclose(got[:, 0], uv[:, 0] * W / 960.0, rtol=1e-6, atol=1e-4)
        assert np.allclose(got[:, 1], uv[:, 1] * H / 540.0, rtol=1e-6, atol=1e-4)
