"""TEST INFRASTRUCTURE (oracle): sphericylindrical-harmonic (SCH) appearance,
the view- and time-dependent colour of 4D Gaussian splatting that the paper
replaces by one RGB value per Gaussian and ablates (Sec. 3.1, the 4D
Gaussian-splatting preliminaries and their SCH equation; Table 2, "SCH" row;
Sec. 4.4, the 4D SCH ablation).  Plain FP64 numpy, shares nothing with the
HIP path.

The basis (Sec. 3.1, SCH equation): Z_{nl}^m(t, d) = cos(2 pi n t / T) Y_l^m(d),
with Y_l^m the real spherical harmonics, orthonormal on the unit sphere:

    Y_{l,0}  = K_l^0 P_l^0(cos th)
    Y_{l,m}  = sqrt(2) K_l^m P_l^m(cos th) cos(m ph)      m > 0
    Y_{l,-m} = sqrt(2) K_l^m P_l^m(cos th) sin(m ph)      m > 0
    K_l^m    = sqrt((2l + 1) / (4 pi) (l - m)! / (l + m)!)

where P_l^m is the associated Legendre function without the Condon-Shortley
phase (P_1^1(x) = +sqrt(1 - x^2)), th the polar angle from +z and ph the
azimuth from +x towards +y.  The paper gives neither the degrees nor the
phase convention; these are readings (degree L <= 3 and frequencies
n = 0..N, N <= 2, chosen by the caller; T the period in view-time units).

Basis index b = n (L + 1)^2 + l^2 + l + m.  Coefficients [3 K, n_gauss]
with row b * 3 + c (c = R, G, B), K = (N + 1)(L + 1)^2.  The colour of a
Gaussian seen by a view at time t is

    colour_c = sum_b coef[b * 3 + c] Z_b(t, d),  d = (mu_c - C) / |mu_c - C|,

with mu_c the Gaussian's conditional mean at t (Sec. 3.3, Eq. "4dgs") and C
the camera centre.  With L = N = 0 it is Y_00 coef_c = coef_c / (2 sqrt(pi)),
a constant RGB value.
"""
from __future__ import annotations

import math

import numpy as np

from . import _views


def n_basis(L: int, N: int) -> int:
    return (N + 1) * (L + 1) ** 2


def _assoc_legendre(l_max: int, x):
    """P_l^m(x), no Condon-Shortley phase, for 0 <= m <= l <= l_max, by the
    standard recurrences: P_m^m = (2m - 1)!! (1 - x^2)^(m/2),
    P_{m+1}^m = x (2m + 1) P_m^m,
    (l - m) P_l^m = x (2l - 1) P_{l-1}^m - (l + m - 1) P_{l-2}^m."""
    x = np.asarray(x, np.float64)
    s = np.sqrt(np.maximum(0.0, 1.0 - x * x))
    P = {}
    for m in range(l_max + 1):
        dfact = 1.0
        for k in range(1, 2 * m, 2):
            dfact *= k
        P[(m, m)] = dfact * s ** m
        if m + 1 <= l_max:
            P[(m + 1, m)] = x * (2 * m + 1) * P[(m, m)]
        for l in range(m + 2, l_max + 1):
            P[(l, m)] = (x * (2 * l - 1) * P[(l - 1, m)] - (l + m - 1) * P[(l - 2, m)]) / (l - m)
    return P


def real_sh(L: int, d):
    """Real spherical harmonics up to degree L at directions d [..., 3]
    (normalised here): [..., (L + 1)^2], index l^2 + l + m."""
    d = np.asarray(d, np.float64)
    d = d / np.linalg.norm(d, axis=-1, keepdims=True)
    x, y, z = d[..., 0], d[..., 1], d[..., 2]
    ph = np.arctan2(y, x)
    P = _assoc_legendre(L, z)
    out = np.zeros(d.shape[:-1] + ((L + 1) ** 2,))
    for l in range(L + 1):
        for m in range(l + 1):
            K = math.sqrt((2 * l + 1) / (4 * math.pi) * math.factorial(l - m) / math.factorial(l + m))
            if m == 0:
                out[..., l * l + l] = K * P[(l, 0)]
            else:
                out[..., l * l + l + m] = math.sqrt(2.0) * K * P[(l, m)] * np.cos(m * ph)
                out[..., l * l + l - m] = math.sqrt(2.0) * K * P[(l, m)] * np.sin(m * ph)
    return out


def basis(L: int, N: int, T: float, t, d):
    """Z_b(t, d) [..., K]: the temporal factor cos(2 pi n t / T) times the
    real spherical harmonic, index b = n (L + 1)^2 + l^2 + l + m."""
    Y = real_sh(L, d)
    t = np.asarray(t, np.float64)
    return np.concatenate([np.cos(2.0 * math.pi * n * t / T)[..., None] * Y
                           for n in range(N + 1)], axis=-1)


def camera_centres(views):
    """Camera centres C = -R^T t of views [V, 23] (world -> camera x_c = R x + t)."""
    v = _views(views)
    R = v[:, 0:12].reshape(-1, 3, 4)[:, :, :3]
    tr = v[:, 0:12].reshape(-1, 3, 4)[:, :, 3]
    return -np.einsum("vij,vi->vj", R, tr)


def colour(coef, mu3, views, L, N, T):
    """RGB [V, n, 3] of every (view, Gaussian) from coefficients [3 K, n] and
    conditional means mu3 [V, n, 3] (at each view's time)."""
    v = _views(views)
    K = n_basis(L, N)
    C = np.asarray(coef, np.float64).reshape(K, 3, -1)
    Cc = camera_centres(v)
    out = np.zeros(mu3.shape)
    for vi in range(v.shape[0]):
        Z = basis(L, N, T, v[vi, 18], mu3[vi] - Cc[vi])      # [n, K]
        out[vi] = np.einsum("gb,bcg->gc", Z, C)
    return out


def backward(coef, mu3, views, L, N, T, grad_rgb, touched=None, h=1e-6):
    """Chain rule of colour(): from grad_rgb [V, n, 3] to
    dcoef [3 K, n] (summed over views; colour is linear in the
    coefficients, so it is grad_rgb times the basis) and
    gmu3 [V, n, 3] = d loss / d mu_c through the viewing direction, by
    central differences of sum_c grad_c colour_c in the unnormalised
    direction v = mu_c - C (step h |v|; the basis normalises v itself).
    Entries with touched == 0 contribute nothing."""
    v = _views(views)
    K = n_basis(L, N)
    C = np.asarray(coef, np.float64).reshape(K, 3, -1)
    Cc = camera_centres(v)
    V, n, _ = mu3.shape
    dcoef = np.zeros((K, 3, n))
    gmu3 = np.zeros((V, n, 3))
    for vi in range(V):
        g = np.asarray(grad_rgb[vi], np.float64)
        if touched is not None:
            g = g * (np.asarray(touched[vi]) > 0)[:, None]
        dvec = mu3[vi] - Cc[vi]
        Z = basis(L, N, T, v[vi, 18], dvec)
        dcoef += np.einsum("gb,gc->bcg", Z, g)
        w = np.einsum("bcg,gc->gb", C, g)                      # per-basis weight
        step = h * np.linalg.norm(dvec, axis=-1)
        for j in range(3):
            e = np.zeros(3)
            e[j] = 1.0
            fp = (basis(L, N, T, v[vi, 18], dvec + step[:, None] * e) * w).sum(-1)
            fm = (basis(L, N, T, v[vi, 18], dvec - step[:, None] * e) * w).sum(-1)
            gmu3[vi, :, j] = (fp - fm) / (2.0 * step)
    return dcoef.reshape(3 * K, n), gmu3


def from_rgb(rgb, L, N):
    """Coefficients [3 K, n] whose colour is the constant rgb [3, n] (only the
    n = 0, l = 0 term: rgb / Y_00)."""
    rgb = np.asarray(rgb, np.float64)
    out = np.zeros((3 * n_basis(L, N), rgb.shape[1]))
    out[0:3] = rgb * (2.0 * math.sqrt(math.pi))
    return out
