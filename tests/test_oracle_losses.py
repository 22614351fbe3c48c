"""Pins for the oracle's losses and optimiser.

* SSIM(x, x) = 1 and SSIM of a constant shift against its closed form;
* SSIM and its gradient against central differences of the oracle's value;
* a known MSE gives a known PSNR;
* Adam: the first steps against a hand-derived closed form (with bias
  correction, the first update is lr * sign(g) for any g != 0).
"""
import numpy as np

from oracle import adam, losses


def test_ssim_identity():
    rng = np.random.default_rng(0)
    x = rng.uniform(0, 1, (3, 20, 23))
    s, g = losses.ssim(x, x)
    assert np.isclose(s, 1.0, rtol=0, atol=1e-14)
    assert np.abs(g).max() < 1e-12


def test_ssim_constant_images_closed_form():
    """Constant images a, b: where the window lies inside the image, mu = a, b
    and all variances vanish, so SSIM = (2ab + C1) / (a^2 + b^2 + C1); at a
    corner the zero padding scales both means by the window mass w inside."""
    a, b = 0.3, 0.7
    x = np.full((1, 31, 31), a)
    y = np.full((1, 31, 31), b)
    S = losses.ssim_map(x, y)
    assert np.isclose(S[0, 15, 15], (2 * a * b + losses.C1) / (a * a + b * b + losses.C1), rtol=1e-12)
    g = losses.gaussian_window()
    w = g[5:, 5:].sum()
    # corner: mu_x = w a, E[x^2] = w a^2 -> var = w(1-w) a^2, cov = w(1-w) ab
    mx, my = w * a, w * b
    vx, vy, cxy = w * (1 - w) * a * a, w * (1 - w) * b * b, w * (1 - w) * a * b
    ref = ((2 * mx * my + losses.C1) * (2 * cxy + losses.C2)) / (
        (mx * mx + my * my + losses.C1) * (vx + vy + losses.C2))
    assert np.isclose(S[0, 0, 0], ref, rtol=1e-12)


def test_ssim_gradient_fd():
    rng = np.random.default_rng(1)
    x = rng.uniform(0, 1, (2, 13, 15))
    y = rng.uniform(0, 1, (2, 13, 15))
    _, g = losses.ssim(x, y)
    h = 1e-6
    for _ in range(25):
        c, i, j = rng.integers(0, 2), rng.integers(0, 13), rng.integers(0, 15)
        xp = x.copy(); xp[c, i, j] += h
        xm = x.copy(); xm[c, i, j] -= h
        fd = (losses.ssim(xp, y, False)[0] - losses.ssim(xm, y, False)[0]) / (2 * h)
        assert abs(fd - g[c, i, j]) <= 1e-6 * max(abs(fd), 1e-4)


def test_l1_and_scene_loss_gradient_fd():
    rng = np.random.default_rng(2)
    x = rng.uniform(0, 1, (3, 9, 10))
    y = rng.uniform(0, 1, (3, 9, 10))
    _, g = losses.scene_loss(x, y)
    h = 1e-7
    for _ in range(20):
        c, i, j = rng.integers(0, 3), rng.integers(0, 9), rng.integers(0, 10)
        xp = x.copy(); xp[c, i, j] += h
        xm = x.copy(); xm[c, i, j] -= h
        fd = (losses.scene_loss(xp, y)[0] - losses.scene_loss(xm, y)[0]) / (2 * h)
        assert abs(fd - g[c, i, j]) <= 1e-5 * max(abs(fd), 1e-4)


def test_psnr_known_mse():
    x = np.zeros((3, 4, 4))
    y = np.full((3, 4, 4), 0.1)     # MSE = 0.01 -> 20 dB
    assert np.isclose(losses.psnr(x, y), 20.0)


def test_adam_closed_form():
    lr = np.array([0.1])
    p = np.array([[1.0]]); m = np.zeros((1, 1)); v = np.zeros((1, 1))
    # step 1: m = 0.1 g, v = 0.001 g^2 -> mh = g, vh = g^2 -> update lr * sign(g)
    p1, m1, v1 = adam.adam_step(p, np.array([[4.0]]), m, v, 1, lr, eps=0.0)
    assert np.isclose(p1[0, 0], 0.9)
    # step 2 with g = -2: m = 0.9*0.4 - 0.2 = 0.16, v = 0.999*0.016 + 0.001*4 = 0.019984
    p2, m2, v2 = adam.adam_step(p1, np.array([[-2.0]]), m1, v1, 2, lr, eps=0.0)
    mh = 0.16 / (1 - 0.81)
    vh = 0.019984 / (1 - 0.998001)
    assert np.isclose(m2[0, 0], 0.16) and np.isclose(v2[0, 0], 0.019984)
    assert np.isclose(p2[0, 0], 0.9 - 0.1 * mh / np.sqrt(vh))


def test_lr_schedule_endpoints():
    assert np.isclose(adam.lr_schedule(0, 1e-5, 1e-7, 5000), 1e-5)
    assert np.isclose(adam.lr_schedule(5000, 1e-5, 1e-7, 5000), 1e-7)
    assert np.isclose(adam.lr_schedule(2500, 1e-5, 1e-7, 5000), 1e-6)
