"""TEST INFRASTRUCTURE: plain numpy oracle of the map between a 4D
Gaussian's motion -- its velocity v and temporal scale s_t -- and the
rotor-form parameters (log scales, left and right unit quaternions).

The paper's motion-aware reading (Sec. 3.3): sliced at time t, a 4D
Gaussian's conditional mean moves as mu_xyz + Sigma_{xyz,t} Sigma_tt^-1 (t -
mu_t), so its velocity is v = Sigma_{xyz,t} / Sigma_tt, and its temporal
opacity falls off with Sigma_tt = s_t^2.  The learned initialisation
predicts (log s_t, v) and keeps an isotropic spatial scale s, so it needs
the 4D covariance whose conditional has covariance s^2 I, slope v and
temporal variance s_t^2:

    Sigma = [[s^2 I + s_t^2 v v^T, s_t^2 v],
             [s_t^2 v^T,           s_t^2  ]]

(Schur complement: Sigma_c = s^2 I + s_t^2 v v^T - s_t^2 v v^T = s^2 I).
That covariance is written in rotor form by an eigendecomposition (cyclic
Jacobi rotations, FP64) Sigma = R diag(lambda) R^T with det R = +1, scales
sqrt(lambda), and a factorisation of R in SO(4) into a left and a right
unit quaternion: the 16 maps p -> e_a p e_b of the quaternion basis are
orthogonal (each of squared Frobenius norm 4), so the coefficients
<R, L(e_a) R(e_b)> / 4 of R form the rank-one matrix q_l q_r^T (the
associate-matrix construction of Van Elfrinkhof; Perez-Gracia and Thomas,
2017).

Conventions shared with the rasterizer's parameters: the 4D rotation maps
p = t + x i + y j + z k to q_l p q_r; coordinates are ordered (x, y, z, t);
quaternions are (w, x, y, z); log scales are rows 4..7 and the two
quaternions rows 8..15 of the [20, N] parameter planes.

Only ``tests/`` may import this module.
"""
from __future__ import annotations

import numpy as np

# space-time axis (x, y, z, t) <- quaternion basis index (i, j, k, 1)
PERM = (1, 2, 3, 0)


def sigma_from_motion(log_s, log_st, v):
    """The 4D covariance above (x, y, z, t order)."""
    s2 = np.exp(2.0 * float(log_s))
    st2 = np.exp(2.0 * float(log_st))
    v = np.asarray(v, np.float64).reshape(3)
    S = np.zeros((4, 4))
    S[:3, :3] = s2 * np.eye(3) + st2 * np.outer(v, v)
    S[:3, 3] = S[3, :3] = st2 * v
    S[3, 3] = st2
    return S


def motion_from_sigma(S):
    """(log s_t, v) of a 4D covariance: s_t^2 = Sigma_tt, v = Sigma_{xyz,t} / Sigma_tt."""
    S = np.asarray(S, np.float64)
    return 0.5 * np.log(S[3, 3]), S[:3, 3] / S[3, 3]


def jacobi_eigh(A, sweeps=60):
    """Eigenvalues and eigenvectors (columns) of a symmetric matrix by cyclic
    Jacobi rotations (each rotation zeroes one off-diagonal pair), FP64."""
    A = np.array(A, np.float64)
    n = A.shape[0]
    V = np.eye(n)
    for _ in range(sweeps):
        off = np.sqrt(np.sum(np.tril(A, -1) ** 2))
        if off <= 1e-300 or off <= 1e-17 * np.sqrt(np.sum(A * A)):
            break
        for p in range(n - 1):
            for q in range(p + 1, n):
                if A[p, q] == 0.0:
                    continue
                # a negligible A[p, q] makes theta overflow to inf, and t = 0:
                # the identity rotation, the limit of the formula
                with np.errstate(over="ignore"):
                    theta = (A[q, q] - A[p, p]) / (2.0 * A[p, q])
                    t = np.sign(theta) / (abs(theta) + np.hypot(theta, 1.0)) if theta != 0 else 1.0
                c = 1.0 / np.sqrt(t * t + 1.0)
                s = t * c
                J = np.eye(n)
                J[p, p] = J[q, q] = c
                J[p, q] = s
                J[q, p] = -s
                A = J.T @ A @ J
                V = V @ J
    return np.diag(A).copy(), V


def quat_mul(a, b):
    w1, x1, y1, z1 = a
    w2, x2, y2, z2 = b
    return np.array([w1 * w2 - x1 * x2 - y1 * y2 - z1 * z2,
                     w1 * x2 + x1 * w2 + y1 * z2 - z1 * y2,
                     w1 * y2 - x1 * z2 + y1 * w2 + z1 * x2,
                     w1 * z2 + x1 * y2 - y1 * x2 + z1 * w2])


def _basis_map(a, b):
    """4x4 matrix (quaternion basis 1, i, j, k) of p -> a p b."""
    E = np.eye(4)
    return np.stack([quat_mul(quat_mul(a, E[c]), b) for c in range(4)], axis=1)


def rotation_from_rotors(ql, qr):
    """R (x, y, z, t order) of p -> q_l p q_r for unit quaternions."""
    Q = _basis_map(np.asarray(ql, np.float64), np.asarray(qr, np.float64))
    return Q[np.ix_(PERM, PERM)]


def rotors_from_rotation(R):
    """(q_l, q_r) with p -> q_l p q_r equal to R in SO(4) (x, y, z, t order);
    the pair is unique up to a common sign, fixed here by making the
    largest |q_l| component positive."""
    R = np.asarray(R, np.float64)
    Q = np.zeros((4, 4))
    Q[np.ix_(PERM, PERM)] = R
    E = np.eye(4)
    A = np.array([[np.sum(Q * _basis_map(E[a], E[b])) / 4.0 for b in range(4)] for a in range(4)])
    a = int(np.argmax(np.linalg.norm(A, axis=1)))
    ql_a = np.linalg.norm(A[a])
    qr = A[a] / ql_a
    b = int(np.argmax(np.abs(qr)))
    ql = A[:, b] / qr[b]
    return ql / np.linalg.norm(ql), qr / np.linalg.norm(qr)


def rotor_params(S):
    """Log scales [4] (x, y, z, t slots), q_l [4] and q_r [4] with
    (R diag(s)) (R diag(s))^T = S."""
    lam, V = jacobi_eigh(S)
    if np.linalg.det(V) < 0:
        V[:, 0] = -V[:, 0]
    ql, qr = rotors_from_rotation(V)
    return 0.5 * np.log(lam), ql, qr


def init_columns(base, log_st, v):
    """Rotor-form parameter columns from heuristic columns base [20, N]
    (isotropic spatial scale in row 4), predicted log s_t [N] and v [3, N]:
    rows 4..15 replaced, the rest kept."""
    out = np.array(base, np.float64)
    for g in range(out.shape[1]):
        S = sigma_from_motion(out[4, g], log_st[g], v[:, g])
        ls, ql, qr = rotor_params(S)
        out[4:8, g] = ls
        out[8:12, g] = ql
        out[12:16, g] = qr
    return out
