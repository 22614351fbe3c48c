"""Pins for the oracle's back projection and heuristic initialisation
(oracle/init.py; Sec. 3.2 back-projection equation, Sec. 4.1 temporal
scales).

* back projection: projecting each world point with the same camera returns
  its pixel centre and depth (closed form of the pinhole model); a pixel at
  the principal point lands on the optical axis; pixels at or under the
  cover threshold are not kept; order is row-major;
* initialisation, read through the C oracle's covariance and conditional:
  identity rotors give R = I, so the slice at any time has the centroid as
  its mean and diag(s_xyz^2) as its covariance (no motion); o_t = 0.1 at
  the mean timestamp; a dynamic point falls to 0.1 e^-1/2 two frame
  intervals away (s_t = 2 / fps), a static one only a whole video away
  (s_t = 1) and is never culled within the video (255 o_t >= 1); an
  unpruned class takes the footprint of one pixel at its depth.
"""
import numpy as np

from oracle import init as oinit
from paper_2510_01119_amd import synth


def _view():
    Rt = synth.look_at((0.4, -0.3, -2.5), (0.1, 0.0, 0.2))
    return synth.make_view(Rt, 300.0, 280.0, 40.0, 30.0, 80, 60, 0.5)


def test_backprojection_round_trip():
    v = _view()
    rng = np.random.default_rng(0)
    cover = rng.uniform(0.0, 1.0, (60, 80))
    depth = rng.uniform(0.5, 6.0, (60, 80))
    X, D, pix = oinit.backproject(depth * cover, cover, v, 0.5)
    assert np.array_equal(pix, np.nonzero(cover.reshape(-1) > 0.5)[0])
    assert np.all(np.diff(pix) > 0)
    Rt = v[:12].reshape(3, 4)
    xc = Rt[:, :3] @ X + Rt[:, 3:4]
    y, x = np.divmod(pix, 80)
    assert np.allclose(xc[2], D, rtol=1e-12)
    assert np.allclose(v[12] * xc[0] / xc[2] + v[14], x + 0.5, atol=1e-9)
    assert np.allclose(v[13] * xc[1] / xc[2] + v[15], y + 0.5, atol=1e-9)
    assert np.allclose(D, depth.reshape(-1)[pix], rtol=1e-12)


def test_backprojection_principal_axis():
    # identity rotation, camera 3 units behind the origin: the pixel whose
    # centre is the principal point (cx, cy) = (20, 15) lies on the axis
    v = synth.front_view(40, 30, 50.0, 3.0, 0.5)
    cover = np.zeros((30, 40))
    depth = np.zeros((30, 40))
    # pixel centre (x + 1/2, y + 1/2) = (20, 15) is not a pixel centre; use
    # the four pixels around it and check their symmetry instead
    for (y, x) in ((14, 19), (14, 20), (15, 19), (15, 20)):
        cover[y, x] = 1.0
        depth[y, x] = 2.0
    X, D, pix = oinit.backproject(depth, cover, v, 0.5)
    assert len(pix) == 4
    assert np.allclose(X[2], -1.0) and np.allclose(D, 2.0)
    assert np.allclose(X[:2].sum(axis=1), 0.0, atol=1e-12)
    assert np.allclose(np.abs(X[0]), 0.5 / 50.0 * 2.0)


def test_cover_threshold_is_strict():
    v = synth.front_view(8, 4, 10.0, 3.0, 0.5)
    cover = np.full((4, 8), 0.5)
    cover[1, 3] = 0.5000001
    _, _, pix = oinit.backproject(np.ones((4, 8)), cover, v, 0.5)
    assert pix.tolist() == [1 * 8 + 3]


def test_heuristic_init_meaning(oracle_lib):
    rng = np.random.default_rng(1)
    k, frames, vs, vd = 40, 200, 0.01, 0.004
    xyz = rng.uniform(-1, 1, (3, k))
    rgb = rng.uniform(0, 1, (3, k))
    t = rng.uniform(0, 1, k)
    dyn = np.arange(k) % 2 == 1
    p = oinit.heuristic_init(xyz, rgb, t, dyn, vs, vd, frames)
    for g in range(k):
        S = oracle_lib.covariance(p, g)
        s = vd if dyn[g] else vs
        st = 2.0 / frames if dyn[g] else 1.0
        assert np.allclose(S, np.diag([s * s] * 3 + [st * st]), rtol=1e-12, atol=0)
        for dt in (0.0, 0.37 * st):
            mu, Sc, ot = oracle_lib.conditional(p, g, t[g] + dt)
            assert np.allclose(mu, xyz[:, g], rtol=0, atol=1e-15)          # no motion
            assert np.allclose(Sc, np.diag([s * s] * 3), rtol=1e-12, atol=0)
            assert np.isclose(ot, 0.1 * np.exp(-0.5 * (dt / st) ** 2), rtol=1e-12)
        # one temporal scale away: o e^-1/2 (two frame intervals for a
        # dynamic point, the whole video for a static one)
        _, _, ot = oracle_lib.conditional(p, g, t[g] + st)
        assert np.isclose(ot, 0.1 * np.exp(-0.5), rtol=1e-12)
        if not dyn[g]:
            for tt in np.linspace(0.0, 1.0, 11):
                assert 255.0 * oracle_lib.conditional(p, g, tt)[2] >= 1.0
    assert np.allclose(p[17:20], rgb) and np.allclose(p[3], t)


def test_heuristic_init_unpruned_class():
    k = 6
    depth = np.linspace(1.0, 3.0, k)
    dyn = np.array([0, 1, 0, 1, 0, 1], bool)
    p = oinit.heuristic_init(np.zeros((3, k)), np.zeros((3, k)), np.zeros(k), dyn, 0.02, 0.0, 100,
                             depth=depth, focal=500.0)
    assert np.allclose(np.exp(p[4, dyn]), depth[dyn] / 500.0)
    assert np.allclose(np.exp(p[4, ~dyn]), 0.02)
