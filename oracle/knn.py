"""TEST INFRASTRUCTURE: brute-force oracle of the point-cloud features of
the learned initialisation.

* k nearest neighbours: for each point, the k other points of smallest
  Euclidean distance (FP64), ties by smaller index; a point is never its
  own neighbour (duplicates at the same position are other points).
* features, 16 per point, in this order:
    0-2   position xyz (the voxel centroid after grid pruning, Sec. 3.2)
    3     mean camera depth of the back-projected pixels of the voxel
    4     mean 2D optical-flow magnitude of those pixels (pixels per frame)
    5-7   mean of the offsets x_nbr - x over the 8 neighbours
    8-10  variance (population, per axis) of those offsets
    11-13 mean colour
    14    mean timestamp (normalised to [0, 1])
    15    motion class (1 dynamic, 0 static)
  then standardised: (f - shift) * scale per feature.
The pruned-point attributes averaged per voxel are those the grid pruning
of Sec. 3.2 carries (colour, timestamp, motion probability) plus depth and
flow magnitude.

Only ``tests/`` may import this module.
"""
from __future__ import annotations

import numpy as np

K = 8
N_FEATURES = 16


def knn(xyz, k=K, queries=None, chunk=2048):
    """Neighbour ids [len(queries), k] and squared distances, FP64."""
    X = np.asarray(xyz, np.float64).T            # [N, 3]
    n = X.shape[0]
    q = np.arange(n) if queries is None else np.asarray(queries)
    ids = np.zeros((len(q), k), np.int64)
    d2s = np.zeros((len(q), k))
    idx = np.arange(n)
    for s in range(0, len(q), chunk):
        qq = q[s:s + chunk]
        d2 = ((X[None, :, :] - X[qq][:, None, :]) ** 2).sum(axis=2)
        for r, i in enumerate(qq):
            row = d2[r].copy()
            row[i] = np.inf
            order = np.lexsort((idx, row))[:k]
            ids[s + r] = order
            d2s[s + r] = row[order]
    return ids, d2s


def features(xyz, depth, flow, rgb, t, dyn, nbr):
    """Raw (unstandardised) features [16, N] from pruned points (xyz [3, N],
    depth [N], flow [N], rgb [3, N], t [N], dyn [N]) and their neighbour
    ids nbr [N, 8]."""
    X = np.asarray(xyz, np.float64)
    off = X[:, nbr] - X[:, :, None]                 # [3, N, 8]
    mean = off.mean(axis=2)
    var = ((off - mean[:, :, None]) ** 2).mean(axis=2)
    F = np.zeros((N_FEATURES, X.shape[1]))
    F[0:3] = X
    F[3] = depth
    F[4] = flow
    F[5:8] = mean
    F[8:11] = var
    F[11:14] = rgb
    F[14] = t
    F[15] = np.asarray(dyn, np.float64)
    return F


def standardise(F, shift, scale):
    return (np.asarray(F, np.float64) - np.asarray(shift, np.float64)[:, None]) \
        * np.asarray(scale, np.float64)[:, None]
