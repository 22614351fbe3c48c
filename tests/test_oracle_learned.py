"""Pins of the learned-initialisation oracle (network, motion <-> rotor
map, neighbour features) to things other than itself: library conversions
and eigen-solvers, hand-evaluated special cases, closed-form lattices and
central differences."""
import math

import numpy as np
import pytest
import torch

import oracle
from oracle import knn as K
from oracle import mlp as M
from oracle import motion as MO


# ---------------------------------------------------------------- network
def test_param_count():
    assert M.N_PARAMS == 9668


def test_bf16_round_matches_torch():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.standard_normal(20000).astype(np.float32) * 10.0 ** rng.integers(-6, 6, 20000),
                        np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, 1.0 + 2 ** -8 + 2 ** -20,
                                  -2.5, 0.0, -0.0, 65504.0, 1e-40], np.float32)]).astype(np.float32)
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float32).numpy()
    got = M.bf16_round(x)
    assert np.array_equal(got.view(np.uint32), ref.view(np.uint32))
    # ties to even: 1 + 2^-8 is halfway between 1 and 1 + 2^-7 -> 1
    assert got[20001] == 1.0 and got[20002] == np.float32(1.0 + 2 ** -6)
    assert got[20003] == np.float32(1.0 + 2 ** -7)


def test_silu_special_values():
    assert M.silu(np.array(0.0)) == 0.0
    assert abs(M.dsilu(np.array(0.0)) - 0.5) < 1e-15
    z = np.linspace(-8, 8, 33)
    h = 1e-6
    assert np.allclose(M.dsilu(z), (M.silu(z + h) - M.silu(z - h)) / (2 * h), atol=1e-9)
    assert abs(M.silu(np.array(1.0)) - 1.0 / (1.0 + math.exp(-1.0))) < 1e-15


def test_zero_weights_give_last_bias():
    rng = np.random.default_rng(1)
    theta = np.zeros(M.N_PARAMS)
    for (W, b) in M.unpack(theta):
        b[:] = rng.standard_normal(b.shape)
    y, _ = M.forward(theta, rng.standard_normal((5, 16)))
    assert np.array_equal(y, np.broadcast_to(M.unpack(theta)[3][1], (5, 4)))


def test_single_unit_chain_by_hand():
    """Only unit 0 of each hidden layer is wired: y_k = c_k h3 + d_k with
    h3 = silu(-h2), h2 = silu(1.5 h1 + 0.25), h1 = silu(2 x_3 + 0.5)."""
    theta = np.zeros(M.N_PARAMS)
    L = M.unpack(theta)
    L[0][0][0, 3] = 2.0
    L[0][1][0] = 0.5
    L[1][0][0, 0] = 1.5
    L[1][1][0] = 0.25
    L[2][0][0, 0] = -1.0
    c = np.array([1.0, -2.0, 3.0, 0.5])
    d = np.array([0.1, 0.2, -0.3, 0.0])
    L[3][0][:, 0] = c
    L[3][1][:] = d
    x = np.zeros((1, 16))
    x[0, 3] = 0.7

    def s(z):
        return z / (1.0 + math.exp(-z))
    h3 = s(-s(1.5 * s(2 * 0.7 + 0.5) + 0.25))
    y, _ = M.forward(theta, x)
    assert np.allclose(y[0], c * h3 + d, rtol=0, atol=1e-15)


def test_backward_central_differences():
    rng = np.random.default_rng(2)
    theta = M.bf16_round(rng.standard_normal(M.N_PARAMS).astype(np.float32) * 0.2).astype(np.float64)
    X = rng.standard_normal((7, 16))
    dY = rng.standard_normal((7, 4))
    g, gx = M.backward(theta, X, dY)

    def L(th, x):
        return float((M.forward(th, x)[0] * dY).sum())
    h = 1e-6
    for k in rng.choice(M.N_PARAMS, 60, replace=False):
        e = np.zeros(M.N_PARAMS)
        e[k] = h
        fd = (L(theta + e, X) - L(theta - e, X)) / (2 * h)
        assert abs(fd - g[k]) <= 1e-7 * max(1.0, abs(fd)), k
    for (i, j) in [(0, 0), (3, 15), (6, 7), (2, 11)]:
        e = np.zeros_like(X)
        e[i, j] = h
        fd = (L(theta, X + e) - L(theta, X - e)) / (2 * h)
        assert abs(fd - gx[i, j]) <= 1e-7 * max(1.0, abs(fd))


# ---------------------------------------------------------------- motion map
def test_jacobi_against_library():
    rng = np.random.default_rng(3)
    for _ in range(20):
        B = rng.standard_normal((4, 4))
        A = B @ B.T + np.diag(rng.uniform(0, 1, 4))
        lam, V = MO.jacobi_eigh(A)
        assert np.allclose(V @ np.diag(lam) @ V.T, A, atol=1e-12 * np.abs(A).max())
        assert np.allclose(V.T @ V, np.eye(4), atol=1e-13)
        assert np.allclose(np.sort(lam), np.linalg.eigvalsh(A), rtol=1e-12)


def _rand_quat(rng):
    q = rng.standard_normal(4)
    return q / np.linalg.norm(q)


def test_rotation_matches_c_oracle():
    """R diag(s^2) R^T from this module's rotor map equals the C oracle's
    covariance for the same raw parameters."""
    rng = np.random.default_rng(4)
    for _ in range(20):
        p = np.zeros((20, 1))
        p[4:8, 0] = rng.normal(-1, 0.5, 4)
        ql, qr = _rand_quat(rng), _rand_quat(rng)
        p[8:12, 0], p[12:16, 0] = ql, qr
        R = MO.rotation_from_rotors(ql, qr)
        s = np.exp(p[4:8, 0])
        assert np.allclose(R.T @ R, np.eye(4), atol=1e-14)
        assert abs(np.linalg.det(R) - 1.0) < 1e-13
        S = R @ np.diag(s * s) @ R.T
        assert np.allclose(oracle.covariance(p, 0), S, atol=1e-14)


def test_rotor_factorisation_roundtrip():
    rng = np.random.default_rng(5)
    for _ in range(50):
        ql, qr = _rand_quat(rng), _rand_quat(rng)
        a, b = MO.rotors_from_rotation(MO.rotation_from_rotors(ql, qr))
        sgn = np.sign(np.dot(a, ql))
        assert np.allclose(sgn * a, ql, atol=1e-12) and np.allclose(sgn * b, qr, atol=1e-12)
    # x-t plane rotation by theta: q_l = q_r = (cos theta/2, sin theta/2, 0, 0)
    th = 0.7
    q = np.array([math.cos(th / 2), math.sin(th / 2), 0, 0])
    R = MO.rotation_from_rotors(q, q)
    assert np.allclose(R[[0, 3]][:, [0, 3]], [[math.cos(th), math.sin(th)], [-math.sin(th), math.cos(th)]],
                       atol=1e-15)


@pytest.mark.parametrize("seed", range(6))
def test_motion_roundtrip_through_c_oracle(seed):
    """Sigma(s, s_t, v) -> rotor parameters -> the C oracle's covariance and
    conditional: the covariance comes back, the conditional mean moves with
    slope v, the conditional covariance is s^2 I and Var(t) = s_t^2."""
    rng = np.random.default_rng(100 + seed)
    log_s, log_st = rng.normal(-4.5, 0.3), rng.normal(-2.0, 1.0)
    v = rng.normal(0, 0.5, 3) * (0 if seed == 0 else 1)
    S = MO.sigma_from_motion(log_s, log_st, v)
    ls, ql, qr = MO.rotor_params(S)
    p = np.zeros((20, 1))
    p[0:3, 0] = rng.uniform(-1, 1, 3)
    p[3, 0] = 0.5
    p[4:8, 0], p[8:12, 0], p[12:16, 0] = ls, ql, qr
    p[16, 0] = 2.0
    S2 = oracle.covariance(p, 0)
    assert np.allclose(S2, S, rtol=0, atol=1e-10 * np.abs(S).max())
    lst2, v2 = MO.motion_from_sigma(S2)
    assert abs(lst2 - log_st) < 1e-9 and np.allclose(v2, v, atol=1e-8 * max(1, np.abs(v).max()))
    t1, t2 = 0.45, 0.6
    m1, C1, _ = oracle.conditional(p, 0, t1)
    m2, C2, _ = oracle.conditional(p, 0, t2)
    assert np.allclose((m2 - m1) / (t2 - t1), v, atol=1e-8 * max(1, np.abs(v).max()))
    s2 = math.exp(2 * log_s)
    assert np.allclose(C1, s2 * np.eye(3), atol=1e-9 * s2)


def test_motion_zero_velocity_scales():
    S = MO.sigma_from_motion(-4.0, -1.0, np.zeros(3))
    ls, _, _ = MO.rotor_params(S)
    assert np.allclose(np.sort(ls), np.sort([-4.0, -4.0, -4.0, -1.0]), atol=1e-12)


# ---------------------------------------------------------------- neighbours
def test_knn_cube_corners_closed_form():
    h = 0.02
    corners = np.array([[x, y, z] for x in (-h / 2, h / 2) for y in (-h / 2, h / 2) for z in (-h / 2, h / 2)])
    far = np.array([[1.0, 0, 0], [0, 1.0, 0], [0, 0, -1.0]])
    X = np.concatenate([far[:1], corners, [[0.0, 0.0, 0.0]], far[1:]]).T    # centre at index 9
    ids, d2 = K.knn(X, queries=[9])
    assert sorted(ids[0].tolist()) == list(range(1, 9))
    assert np.allclose(d2[0], 3 * (h / 2) ** 2, rtol=1e-15)
    F = K.features(X, np.zeros(12), np.zeros(12), np.zeros(12), np.zeros(12), K.knn(X)[0])
    assert np.allclose(F[5:8, 9], 0.0, atol=1e-18)
    assert np.allclose(F[8:11, 9], (h / 2) ** 2, rtol=1e-12)


def test_knn_lattice_ties_by_index():
    h = 0.1
    g = np.arange(5) * h
    X = np.array(np.meshgrid(g, g, g, indexing="ij")).reshape(3, -1)
    c = 2 * 25 + 2 * 5 + 2                      # interior point (2, 2, 2)
    ids, d2 = K.knn(X, queries=[c])
    assert np.allclose(d2[0][:6], h * h) and np.allclose(d2[0][6:], 2 * h * h)
    faces = sorted([c - 25, c + 25, c - 5, c + 5, c - 1, c + 1])
    assert sorted(ids[0][:6].tolist()) == faces
    edges = sorted(c + a * 25 + b * 5 + e for a in (-1, 0, 1) for b in (-1, 0, 1) for e in (-1, 0, 1)
                   if abs(a) + abs(b) + abs(e) == 2)
    assert ids[0][6:].tolist() == edges[:2]


def test_knn_against_kdtree():
    from scipy.spatial import cKDTree
    rng = np.random.default_rng(6)
    X = rng.uniform(-1, 1, (3, 3000))
    ids, d2 = K.knn(X)
    dd, _ = cKDTree(X.T).query(X.T, k=9)
    assert np.allclose(np.sqrt(d2), dd[:, 1:], rtol=1e-12)


def test_features_missing_neighbours():
    X = np.array([[0.0, 1.0, 3.0], [0.0, 0.0, 0.0], [0.0, 0.0, 0.0]])
    nbr = np.array([[1, 2, -1, -1, -1, -1, -1, -1], [-1] * 8, [0, -1, -1, -1, -1, -1, -1, -1]])
    t = np.array([0.5, 0.25, 1.0])
    F = K.features(X, np.zeros(3), np.zeros(3), t, np.zeros(3), nbr)
    # point 0: offsets 1 and 3 at time offsets -0.25 and +0.5 -> mean 2,
    # variance 1, time-offset mean 0.125 and variance 0.140625, covariance
    # ((1 - 2)(-0.25 - 0.125) + (3 - 2)(0.5 - 0.125)) / 2 = 0.375; point 1:
    # no neighbour -> all offset statistics 0; point 2: one neighbour ->
    # mean -3, every (co)variance 0
    assert np.allclose(F[5:8, 0], [2, 0, 0]) and np.allclose(F[8:11, 0], [1, 0, 0])
    assert np.allclose(F[11:14, 0], [0.375, 0, 0]) and np.isclose(F[14, 0], 0.140625)
    assert np.all(F[5:15, 1] == 0)
    assert np.allclose(F[5:8, 2], [-3, 0, 0]) and np.all(F[8:15, 2] == 0)


def test_features_trail_slope_is_the_velocity():
    """Neighbours on a trail x = x0 + v (t - t0) (points of one moving
    surface back-projected at different frames): the space-time covariance
    over the time-offset variance is v exactly, for any spacing in time;
    static neighbours (v = 0) give covariance 0."""
    rng = np.random.default_rng(4)
    v = np.array([0.3, -0.1, 0.05])
    tt = np.sort(rng.uniform(0, 1, 9))
    X = (np.array([0.2, 0.1, -0.4])[:, None] + v[:, None] * (tt - tt[4])[None])
    ids, _ = K.knn(X, queries=[4])
    F = K.features(X, np.zeros(9), np.zeros(9), tt, np.ones(9), np.tile(ids, (9, 1)))
    assert sorted(ids[0].tolist()) == [0, 1, 2, 3, 5, 6, 7, 8]
    assert np.allclose(F[11:14, 4] / F[14, 4], v, rtol=1e-12)
    assert np.allclose(F[14, 4], np.var(tt[ids[0]] - tt[4]), rtol=1e-12)
    Xs = np.tile(X[:, 4:5], (1, 9)) + rng.normal(0, 1e-3, (3, 9))
    Fs = K.features(Xs, np.zeros(9), np.zeros(9), tt, np.zeros(9), np.tile(ids, (9, 1)))
    assert np.all(np.abs(Fs[11:14, 4]) < 1e-3 * np.sqrt(Fs[14, 4]) * 3)
