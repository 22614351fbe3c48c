"""TEST INFRASTRUCTURE: brute-force oracle of the point-cloud features of
the learned initialisation.

* k nearest neighbours: for each point, the k other points of smallest
  Euclidean distance (FP64), ties by smaller index; a point is never its
  own neighbour (duplicates at the same position are other points).
* features, 16 per point, in this order:
    0-2   position xyz (the voxel centroid after grid pruning, Sec. 3.2)
    3     mean camera depth of the back-projected pixels of the voxel
    4     mean 2D optical-flow magnitude of those pixels (pixels per frame)
    5-7   mean of the spatial offsets x_nbr - x over the 8 neighbours
    8-10  variance (population, per axis) of those offsets
    11-13 covariance (population) of each spatial offset with the time
          offset t_nbr - t (the neighbours' mean timestamps against the
          point's)
    14    variance (population) of the time offsets
    15    motion class (1 dynamic, 0 static)
  then standardised: (f - shift) * scale per feature.  Features 5-14 are
  the mean and (co)variances of the neighbours' space-time offsets; for
  points on a trail x = x0 + v (t - t0), features 11-13 over feature 14 are
  the slope v (a least-squares regression of offset on time).
The pruned-point attributes averaged per voxel are those the grid pruning
of Sec. 3.2 carries (timestamp, motion probability) plus depth and
optical-flow magnitude.

Only ``tests/`` may import this module.
"""
from __future__ import annotations

import numpy as np

K = 8
N_FEATURES = 16


def knn(xyz, k=K, queries=None, chunk=None):
    """Neighbour ids [len(queries), k] and squared distances, FP64."""
    X = np.asarray(xyz, np.float64).T            # [N, 3]
    n = X.shape[0]
    q = np.arange(n) if queries is None else np.asarray(queries)
    ids = np.full((len(q), k), -1, np.int64)
    d2s = np.full((len(q), k), np.inf)
    chunk = chunk or max(1, min(2048, 4_000_000 // max(n, 1)))
    kk = min(k, n - 1)
    if kk <= 0:
        return ids, d2s
    for s in range(0, len(q), chunk):
        qq = q[s:s + chunk]
        d2 = ((X[None, :, :] - X[qq][:, None, :]) ** 2).sum(axis=2)
        d2[np.arange(len(qq)), qq] = np.inf
        thr = np.partition(d2, kk - 1, axis=1)[:, kk - 1]
        for r in range(len(qq)):
            cand = np.nonzero(d2[r] <= thr[r])[0]          # every tie at the k-th distance
            order = cand[np.lexsort((cand, d2[r, cand]))][:kk]
            ids[s + r, :kk] = order
            d2s[s + r, :kk] = d2[r, order]
    return ids, d2s


def features(xyz, depth, flow, t, dyn, nbr):
    """Raw (unstandardised) features [16, N] from pruned points (xyz [3, N],
    depth [N], flow [N], timestamps t [N], dyn [N]) and their neighbour ids
    nbr [N, 8] (-1 = no neighbour; with none, every offset statistic is 0)."""
    X = np.asarray(xyz, np.float64)
    T = np.asarray(t, np.float64)
    nbr = np.asarray(nbr)
    ok = nbr >= 0                                   # missing neighbours (-1) are skipped
    cnt = ok.sum(axis=1)
    j = np.where(ok, nbr, 0)
    off = np.where(ok[None], X[:, j] - X[:, :, None], 0.0)            # [3, N, 8]
    offt = np.where(ok, T[j] - T[:, None], 0.0)                        # [N, 8]
    den = np.maximum(cnt, 1)
    mean = off.sum(axis=2) / den
    meant = offt.sum(axis=1) / den
    dx = np.where(ok[None], off - mean[:, :, None], 0.0)
    dt = np.where(ok, offt - meant[:, None], 0.0)
    F = np.zeros((N_FEATURES, X.shape[1]))
    F[0:3] = X
    F[3] = depth
    F[4] = flow
    F[5:8] = mean
    F[8:11] = (dx * dx).sum(axis=2) / den
    F[11:14] = (dx * dt[None]).sum(axis=2) / den
    F[14] = (dt * dt).sum(axis=1) / den
    F[15] = np.asarray(dyn, np.float64)
    return F


def standardise(F, shift, scale):
    return (np.asarray(F, np.float64) - np.asarray(shift, np.float64)[:, None]) \
        * np.asarray(scale, np.float64)[:, None]
