"""Pins for the oracle's 4D covariance and its conditional at time t
(Sec. 3.3, Eq. "4dgs"; motion-aware opacity o_t = o N(t; mu_4, Sigma_44)).

* rotor invariants: Sigma = R S^2 R^T has eigenvalues s^2 for any unit pair;
* special cases: identity rotors give diag(s^2); q_r = conj(q_l) is the
  textbook 3D quaternion rotation (scipy) with the time axis fixed; equal
  rotors about i rotate the x-t plane, whose conditional variance and
  velocity have a closed form;
* self-check (ii): the conditional mean, covariance and temporal falloff
  against brute-force numerical marginalisation of the 4D density on a grid.
"""
import numpy as np
import pytest
from scipy.spatial.transform import Rotation


def _one(mean=(0.1, -0.2, 0.3, 0.4), ls=(-1.0, -1.5, -0.7, -1.2), ql=(1, 0, 0, 0),
         qr=(1, 0, 0, 0), logit=0.3, rgb=(0.2, 0.5, 0.9)):
    p = np.zeros((20, 1))
    p[0:4, 0] = mean
    p[4:8, 0] = ls
    p[8:12, 0] = ql
    p[12:16, 0] = qr
    p[16, 0] = logit
    p[17:20, 0] = rgb
    return p


def test_identity_rotors_give_diagonal(oracle_lib):
    ls = np.array([-1.0, -1.5, -0.7, -1.2])
    S = oracle_lib.covariance(_one(ls=ls), 0)
    assert np.allclose(S, np.diag(np.exp(2 * ls)), rtol=1e-14, atol=0)


def test_eigenvalues_are_squared_scales(oracle_lib):
    rng = np.random.default_rng(3)
    for _ in range(50):
        ls = rng.normal(-1, 0.7, 4)
        ql = rng.standard_normal(4) * rng.uniform(0.3, 3.0)   # un-normalised on purpose
        qr = rng.standard_normal(4) * rng.uniform(0.3, 3.0)
        S = oracle_lib.covariance(_one(ls=ls, ql=ql, qr=qr), 0)
        assert np.allclose(S, S.T, atol=1e-15)
        ev = np.sort(np.linalg.eigvalsh(S))
        assert np.allclose(ev, np.sort(np.exp(2 * ls)), rtol=1e-11)


def test_conjugate_pair_is_spatial_rotation(oracle_lib):
    rng = np.random.default_rng(4)
    for _ in range(20):
        q = rng.standard_normal(4)
        q /= np.linalg.norm(q)
        qc = q * np.array([1, -1, -1, -1])
        ls = rng.normal(-1, 0.5, 4)
        S = oracle_lib.covariance(_one(ls=ls, ql=q, qr=qc), 0)
        R3 = Rotation.from_quat([q[1], q[2], q[3], q[0]]).as_matrix()
        ref = R3 @ np.diag(np.exp(2 * ls[:3])) @ R3.T
        assert np.allclose(S[:3, :3], ref, rtol=1e-12, atol=1e-15)
        assert np.allclose(S[:3, 3], 0.0, atol=1e-15)
        assert np.isclose(S[3, 3], np.exp(2 * ls[3]), rtol=1e-13)


@pytest.mark.parametrize("theta", [0.3, 1.1, -0.7, 2.5])
def test_xt_plane_rotation_closed_form(oracle_lib, theta):
    sx, st = 0.4, 0.15
    ls = (np.log(sx), -1.0, -1.3, np.log(st))
    q = (np.cos(theta / 2), np.sin(theta / 2), 0.0, 0.0)
    mean = (0.2, 0.1, -0.3, 0.5)
    p = _one(mean=mean, ls=ls, ql=q, qr=q)
    S = oracle_lib.covariance(p, 0)
    s2, c2 = np.sin(theta) ** 2, np.cos(theta) ** 2
    # conditional variance of x and velocity dx/dt of a plane rotation
    var_c = sx ** 2 * st ** 2 / (s2 * sx ** 2 + c2 * st ** 2)
    t = 0.8
    mu, Sc, ot = oracle_lib.conditional(p, 0, t)
    assert np.isclose(Sc[0, 0], var_c, rtol=1e-12)
    v = S[0, 3] / S[3, 3]
    assert np.isclose(mu[0], mean[0] + v * (t - mean[3]), rtol=1e-12)
    # rotation by theta in the (t, x) plane: |Sigma_xt| = |sin cos (st^2 - sx^2)|
    assert np.isclose(abs(S[0, 3]), abs(np.sin(theta) * np.cos(theta) * (st ** 2 - sx ** 2)),
                      rtol=1e-12)
    assert np.isclose(mu[1], mean[1]) and np.isclose(mu[2], mean[2])


def test_identities(oracle_lib):
    rng = np.random.default_rng(5)
    for _ in range(20):
        p = _one(ls=rng.normal(-1, 0.5, 4), ql=rng.standard_normal(4), qr=rng.standard_normal(4),
                 mean=rng.uniform(-1, 1, 4), logit=rng.normal())
        S = oracle_lib.covariance(p, 0)
        c = S[3, 3]
        mu, Sc, ot = oracle_lib.conditional(p, 0, rng.uniform(0, 1))
        # Schur complement: det Sigma = Sigma_tt det Sc ; Sc is PSD
        assert np.isclose(np.linalg.det(S), c * np.linalg.det(Sc), rtol=1e-10)
        assert np.all(np.linalg.eigvalsh(Sc) > 0)
        # o_t = o at t = mu_t
        _, _, ot0 = oracle_lib.conditional(p, 0, p[3, 0])
        o = 1 / (1 + np.exp(-p[16, 0]))
        assert np.isclose(ot0, o, rtol=1e-15)


@pytest.mark.parametrize("seed", [11, 12, 13])
def test_conditional_vs_bruteforce_marginalisation(oracle_lib, seed):
    """Self-check (ii): numerically integrate the 4D Gaussian density over a
    3D grid at fixed t; its normalised mean and covariance are the
    conditional, and its mass relative to t = mu_t is o_t / o."""
    rng = np.random.default_rng(seed)
    ls = np.array([-1.2, -1.0, -1.4, -1.1]) + rng.normal(0, 0.1, 4)
    p = _one(ls=ls, ql=rng.standard_normal(4), qr=rng.standard_normal(4),
             mean=(0.05, -0.1, 0.2, 0.5), logit=0.7)
    S = oracle_lib.covariance(p, 0)
    Si = np.linalg.inv(S)
    t = 0.5 + 0.6 * np.sqrt(S[3, 3])
    mu_xyz = p[0:3, 0]

    def moments(tt):
        sd = np.sqrt(np.diag(S)[:3])
        n = 96
        axes = [np.linspace(mu_xyz[k] - 9 * sd[k], mu_xyz[k] + 9 * sd[k], n) for k in range(3)]
        X, Y, Z = np.meshgrid(*axes, indexing="ij")
        d = np.stack([X - mu_xyz[0], Y - mu_xyz[1], Z - mu_xyz[2],
                      np.full_like(X, tt - p[3, 0])], axis=-1)
        q = np.einsum("...i,ij,...j->...", d, Si, d)
        w = np.exp(-0.5 * q)
        dv = np.prod([a[1] - a[0] for a in axes])
        mass = w.sum() * dv
        pts = np.stack([X, Y, Z], axis=-1)
        m = (w[..., None] * pts).sum(axis=(0, 1, 2)) * dv / mass
        dd = pts - m
        C = np.einsum("abci,abcj,abc->ij", dd, dd, w) * dv / mass
        return mass, m, C

    mass_t, m_t, C_t = moments(t)
    mass_0, _, _ = moments(p[3, 0])
    mu, Sc, ot = oracle_lib.conditional(p, 0, t)
    o = 1 / (1 + np.exp(-p[16, 0]))
    assert np.allclose(m_t, mu, rtol=0, atol=1e-6 * np.sqrt(np.trace(Sc)))
    assert np.allclose(C_t, Sc, rtol=1e-6, atol=1e-6 * np.trace(Sc))
    assert np.isclose(mass_t / mass_0, ot / o, rtol=1e-6)


def test_fp32_conditional_is_well_conditioned(oracle_lib):
    """The FP32 instance (the kernel's precision and evaluation order) forms
    the conditional covariance from the rows of R S with the time direction
    projected out.  Against the FP64 plain Schur complement its error stays
    at a few roundoffs of |Sc| for random 4D rotations with s_t up to ~1100
    times s_xyz; the plain Schur complement evaluated in FP32 loses about
    eps (s_t / s_xyz)^2 there, which this bound would catch."""
    rng = np.random.default_rng(0)
    worst, worst_plain = 0.0, 0.0
    for ratio_log in (0.0, 2.0, 4.0, 5.0, 6.0, 7.0):
        for _ in range(100):
            ls = rng.normal(-5.0, 0.5, 3)
            p = _one(mean=rng.uniform(-1, 1, 4), ls=(*ls, ls.mean() + ratio_log),
                     ql=rng.standard_normal(4), qr=rng.standard_normal(4)).astype(np.float32)
            mu64, S64, ot64 = oracle_lib.conditional(p.astype(np.float64), 0, 0.5)
            mu32, S32, ot32 = oracle_lib.conditional_f32(p, 0, 0.5)
            scale = np.abs(S64).max()
            err = np.abs(S32.astype(np.float64) - S64).max() / scale
            assert err < 2e-5, (ratio_log, err)
            assert np.allclose(mu32, mu64, rtol=1e-5, atol=1e-6)
            if ot64 >= 1.0 / 255.0:     # the range where o_t decides visibility
                assert abs(ot32 - ot64) <= 1e-5 * ot64
            worst = max(worst, err)
            if ratio_log == 6.0:
                Sg = oracle_lib.covariance(p.astype(np.float64), 0).astype(np.float32)
                c, a = Sg[3, 3], Sg[:3, 3]
                plain = (Sg[:3, :3] - np.outer(a, a) / c).astype(np.float64)
                worst_plain = max(worst_plain, np.abs(plain - S64).max() / scale)
    assert worst < 2e-5
    assert worst_plain > 1e-3
