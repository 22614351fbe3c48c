"""Pins of the oracle's sphericylindrical-harmonic appearance (Sec. 3.1, SCH
equation) against what mathematics fixes, independently of its code:

* orthonormality of the real spherical harmonics on the sphere (Gauss-Legendre
  in cos(theta) times a uniform azimuth grid, exact for these polynomials);
* agreement with scipy's complex spherical harmonics under the stated real
  convention (a library routine the oracle does not call);
* the addition theorem sum_m Y_lm(a) Y_lm(b) = (2l + 1)/(4 pi) P_l(a . b)
  (numpy's Legendre series);
* textbook values (Y_00 = 1 / (2 sqrt(pi)), the polynomial forms on the axes);
* the temporal factor cos(2 pi n t / T) at quarter periods;
* L = N = 0 is a constant RGB colour (from_rgb inverts it);
* the coefficient gradient against central differences of the colour, and
  the direction gradient against the closed form of the degree-1 band,
  d/dv (v_j / |v|) = (e_j - d d_j) / |v|;
* the preprocess backward's conditional-mean input against central
  differences of the oracle's FP64 conditional mean.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import sch
from paper_2510_01119_amd import synth


def _dirs(n, seed):
    rng = np.random.default_rng(seed)
    d = rng.normal(size=(n, 3))
    return d / np.linalg.norm(d, axis=1, keepdims=True)


@pytest.mark.parametrize("L", [0, 1, 2, 3])
def test_real_sh_orthonormal(L):
    x, wx = np.polynomial.legendre.leggauss(16)          # cos(theta) nodes
    nph = 32
    ph = 2 * np.pi * np.arange(nph) / nph
    X, PH = np.meshgrid(x, ph, indexing="ij")
    s = np.sqrt(1 - X ** 2)
    d = np.stack([s * np.cos(PH), s * np.sin(PH), X], -1).reshape(-1, 3)
    w = (wx[:, None] * np.full(nph, 2 * np.pi / nph)[None, :]).reshape(-1)
    Y = sch.real_sh(L, d)
    G = (Y * w[:, None]).T @ Y
    assert np.abs(G - np.eye((L + 1) ** 2)).max() < 1e-12


def test_real_sh_matches_scipy_complex():
    from scipy import special
    d = _dirs(200, 1)
    th = np.arccos(d[:, 2])
    ph = np.arctan2(d[:, 1], d[:, 0])
    Y = sch.real_sh(3, d)
    sph = getattr(special, "sph_harm_y", None)
    for l in range(4):
        for m in range(-l, l + 1):
            am = abs(m)
            if sph is not None:
                c = sph(l, am, th, ph)
            else:
                c = special.sph_harm(am, l, ph, th)
            # scipy carries the Condon-Shortley phase (-1)^m
            if m == 0:
                ref = c.real
            elif m > 0:
                ref = math.sqrt(2) * (-1) ** m * c.real
            else:
                ref = math.sqrt(2) * (-1) ** am * c.imag
            assert np.abs(Y[:, l * l + l + m] - ref).max() < 1e-12, (l, m)


def test_addition_theorem():
    a, b = _dirs(50, 2), _dirs(50, 3)
    Ya, Yb = sch.real_sh(3, a), sch.real_sh(3, b)
    cosg = (a * b).sum(1)
    for l in range(4):
        sl = slice(l * l, (l + 1) ** 2)
        lhs = (Ya[:, sl] * Yb[:, sl]).sum(1)
        c = np.zeros(l + 1)
        c[l] = 1.0
        rhs = (2 * l + 1) / (4 * np.pi) * np.polynomial.legendre.legval(cosg, c)
        assert np.abs(lhs - rhs).max() < 1e-13


def test_textbook_values():
    ex, ey, ez = np.eye(3)
    Y = sch.real_sh(3, np.stack([ex, ey, ez]))
    assert Y[0, 0] == pytest.approx(0.5 / math.sqrt(math.pi), abs=1e-15)
    assert Y[2, 2] == pytest.approx(math.sqrt(3 / (4 * math.pi)), abs=1e-15)     # Y_1,0 = c z
    assert Y[0, 3] == pytest.approx(math.sqrt(3 / (4 * math.pi)), abs=1e-15)     # Y_1,1 = c x
    assert Y[1, 1] == pytest.approx(math.sqrt(3 / (4 * math.pi)), abs=1e-15)     # Y_1,-1 = c y
    assert Y[2, 6] == pytest.approx(0.5 * math.sqrt(5 / math.pi), abs=1e-15)     # (3z^2-1)
    assert Y[0, 8] == pytest.approx(0.25 * math.sqrt(15 / math.pi), abs=1e-15)   # (x^2-y^2)
    assert Y[0, 15] == pytest.approx(0.25 * math.sqrt(35 / (2 * math.pi)), abs=1e-14)  # x(x^2-3y^2)
    assert Y[1, 9] == pytest.approx(-0.25 * math.sqrt(35 / (2 * math.pi)), abs=1e-14)  # y(3x^2-y^2)
    assert Y[2, 12] == pytest.approx(0.5 * math.sqrt(7 / math.pi), abs=1e-14)    # z(5z^2-3)


def test_temporal_factor():
    d = _dirs(4, 5)
    T = 2.0
    Y = sch.real_sh(1, d)
    Z = sch.basis(1, 2, T, T / 4, d)
    assert np.allclose(Z[:, 0:4], Y, atol=1e-15)            # n = 0
    assert np.abs(Z[:, 4:8]).max() < 1e-15                  # cos(pi/2)
    assert np.allclose(Z[:, 8:12], -Y, atol=1e-15)          # cos(pi)


def test_constant_colour_reduction():
    rng = np.random.default_rng(7)
    n, V = 30, 2
    rgb = rng.uniform(0, 1, (3, n))
    coef = sch.from_rgb(rgb, 0, 0)
    views = np.stack([synth.front_view(32, 32, 30.0, 3.0, t) for t in (0.1, 0.7)])
    mu3 = rng.normal(size=(V, n, 3))
    col = sch.colour(coef, mu3, views, 0, 0, 1.0)
    assert np.abs(col - rgb.T[None]).max() < 1e-15
    # higher bands with zero coefficients change nothing
    big = sch.from_rgb(rgb, 3, 2)
    assert np.abs(sch.colour(big, mu3, views, 3, 2, 1.0) - rgb.T[None]).max() < 1e-15


def _case(seed, n=40, L=3, N=1):
    rng = np.random.default_rng(seed)
    K = sch.n_basis(L, N)
    coef = rng.normal(0, 0.5, (3 * K, n))
    views = np.stack([synth.front_view(32, 32, 30.0, 3.0, t) for t in (0.2, 0.9)])
    mu3 = rng.normal(0, 0.7, (2, n, 3))
    g = rng.normal(size=(2, n, 3))
    return coef, views, mu3, g


def test_coefficient_gradient_vs_central_differences():
    coef, views, mu3, g = _case(11)
    T = 1.5
    dcoef, _ = sch.backward(coef, mu3, views, 3, 1, T, g)
    rng = np.random.default_rng(3)
    for _ in range(20):
        r, k = int(rng.integers(0, coef.shape[0])), int(rng.integers(0, coef.shape[1]))
        h = 1e-4
        cp, cm = coef.copy(), coef.copy()
        cp[r, k] += h
        cm[r, k] -= h
        fd = ((sch.colour(cp, mu3, views, 3, 1, T) - sch.colour(cm, mu3, views, 3, 1, T))
              * g).sum() / (2 * h)
        assert dcoef[r, k] == pytest.approx(fd, rel=1e-9, abs=1e-12)


def test_direction_gradient_closed_form_degree_one():
    coef, views, mu3, g = _case(12, L=1, N=0)
    _, gmu3 = sch.backward(coef, mu3, views, 1, 0, 1.0, g)
    C = sch.camera_centres(views)
    c1 = math.sqrt(3 / (4 * math.pi))
    K = coef.reshape(4, 3, -1)
    for vi in range(2):
        v = mu3[vi] - C[vi]
        r = np.linalg.norm(v, axis=1)
        d = v / r[:, None]
        # Y_1,-1 = c1 y, Y_1,0 = c1 z, Y_1,1 = c1 x: gradient in d of sum_b w_b Y_b
        w = np.einsum("bcg,gc->gb", K, g[vi])
        gd = c1 * np.stack([w[:, 3], w[:, 1], w[:, 2]], 1)
        ref = (gd - d * (gd * d).sum(1, keepdims=True)) / r[:, None]
        assert np.abs(gmu3[vi] - ref).max() < 1e-8 * np.abs(ref).max()


def test_touched_masks_contributions():
    coef, views, mu3, g = _case(13)
    touched = np.ones((2, coef.shape[1]), np.int32)
    touched[1, ::2] = 0
    d1, m1 = sch.backward(coef, mu3, views, 3, 1, 1.0, g, touched)
    g2 = g.copy()
    g2[1, ::2] = 0
    d2, m2 = sch.backward(coef, mu3, views, 3, 1, 1.0, g2)
    assert np.array_equal(d1, d2) and np.array_equal(m1, m2)


def test_preprocess_bwd_conditional_mean_input():
    """d/dparams of sum_v w_v . mu_c(view v) through or_preprocess_bwd_mu
    (grad_rec = 0, grad_mu3 = w) against central differences of the FP64
    conditional mean, for every parameter the mean depends on."""
    p = synth.small_set(12, 4, log_s_xyz=(-1.5, 0.3), log_s_t=(-0.5, 0.2)).astype(np.float64)
    views = np.stack([synth.front_view(64, 64, 64.0, 3.0, t) for t in (0.3, 0.6)])
    rec, _, touched = oracle.preprocess_f64(p, views)
    assert (touched > 0).all()
    rng = np.random.default_rng(5)
    w = rng.normal(size=(2, p.shape[1], 3))
    d = oracle.preprocess_bwd(p, views, np.zeros((2, p.shape[1], 9)), grad_mu3=w)
    h = 1e-6
    for g in range(p.shape[1]):
        for k in range(16):
            q = p.copy()
            q[k, g] += h
            fp = (oracle.conditional_mean_all(q, views) * w).sum()
            q[k, g] -= 2 * h
            fm = (oracle.conditional_mean_all(q, views) * w).sum()
            fd = (fp - fm) / (2 * h)
            assert d[k, g] == pytest.approx(fd, rel=2e-6, abs=2e-8), (k, g)
    # rows the conditional mean does not depend on
    assert np.all(d[16:] == 0.0)
