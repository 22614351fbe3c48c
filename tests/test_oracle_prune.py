"""Pins for the oracle's grid pruning (Sec. 3.2, "Grid Pruning"; per-class
voxel sizes of the Lite/Full presets, Sec. 4.1).

* a Python dict brute force (floor division, centroid, attribute means,
  min_count) gives the same cells, counts and means;
* count conservation (min_count = 1), centroid inside its voxel (convexity),
  idempotence (pruning the output again with min_count = 1 is the identity);
* a class with voxel size <= 0 passes through unpruned.
"""
import math

import numpy as np
import pytest


def _points(m, seed):
    rng = np.random.default_rng(seed)
    xyz = rng.normal(0, 0.05, (3, m)).astype(np.float32)
    xyz[:, : m // 3] += 0.2           # a second cluster, straddling no origin
    attr = rng.uniform(0, 1, (5, m)).astype(np.float32)
    cls = (rng.uniform(0, 1, m) < 0.3).astype(np.uint8)
    return xyz, attr, cls


def _dict_prune(xyz, attr, cls, vs, vd, min_count):
    cells = {}
    m = xyz.shape[1]
    for i in range(m):
        c = int(cls[i]) if cls is not None else 0
        v = vd if c else vs
        if v <= 0:
            key = (c, 1, i)
        else:
            key = (c, 0) + tuple(math.floor(np.float32(xyz[a, i]) / np.float32(v)) for a in range(3))
        cells.setdefault(key, []).append(i)
    out = []
    for key in sorted(cells, key=lambda k: (k[0], k[1], k[2:])):
        idx = cells[key]
        if len(idx) < min_count:
            continue
        out.append((key, len(idx), xyz[:, idx].astype(np.float64).mean(axis=1),
                    attr[:, idx].astype(np.float64).mean(axis=1)))
    return out


@pytest.mark.parametrize("vs,vd,min_count", [(0.02, 0.02, 1), (0.03, 0.01, 2), (0.02, 0.0, 1),
                                             (0.05, 0.05, 4)])
def test_prune_vs_dict(oracle_lib, vs, vd, min_count):
    xyz, attr, cls = _points(3000, 0)
    out = oracle_lib.grid_prune(xyz, attr, cls, vs, vd, min_count)
    ref = _dict_prune(xyz, attr, cls, vs, vd, min_count)
    assert len(ref) == len(out["count"])
    for i, (key, cnt, mx, ma) in enumerate(ref):
        assert out["count"][i] == cnt
        assert np.allclose(out["xyz"][:, i], mx, rtol=1e-6, atol=1e-7)
        assert np.allclose(out["attr"][:, i], ma, rtol=1e-6, atol=1e-7)
        k = int(out["key"][i])
        assert (k >> 63) == key[0]
        assert ((k >> 62) & 1) == key[1]
        if key[1] == 0:
            got = [((k >> 40) & 0xFFFFF) - 524288, ((k >> 20) & 0xFFFFF) - 524288,
                   (k & 0xFFFFF) - 524288]
            assert tuple(got) == key[2:]
        else:
            assert (k & ((1 << 62) - 1)) == key[2]
    assert np.all(np.diff(out["key"].astype(np.uint64)) > 0)


def test_prune_invariants(oracle_lib):
    xyz, attr, cls = _points(5000, 1)
    v = 0.015
    out = oracle_lib.grid_prune(xyz, attr, None, v, v, 1)
    assert out["count"].sum() == xyz.shape[1]
    # centroid lies in its voxel (floor division)
    cells = np.floor(out["xyz"].astype(np.float64) / v)
    k = out["key"].astype(np.uint64)
    ix = ((k >> np.uint64(40)) & np.uint64(0xFFFFF)).astype(np.int64) - 524288
    iy = ((k >> np.uint64(20)) & np.uint64(0xFFFFF)).astype(np.int64) - 524288
    iz = (k & np.uint64(0xFFFFF)).astype(np.int64) - 524288
    for a, ia in enumerate((ix, iy, iz)):
        # allow one-ulp slack for a centroid that lands on a cell face
        assert np.all((cells[a] == ia) | (np.abs(out["xyz"][a] - ia * v) < 1e-6)
                      | (np.abs(out["xyz"][a] - (ia + 1) * v) < 1e-6))
    # idempotence
    again = oracle_lib.grid_prune(out["xyz"], out["attr"], None, v, v, 1)
    assert np.array_equal(again["key"], out["key"])
    assert np.all(again["count"] == 1)
    assert np.array_equal(again["xyz"], out["xyz"])


def test_floor_not_truncation(oracle_lib):
    xyz = np.array([[-0.004, 0.004], [0.0, 0.0], [0.0, 0.0]], np.float32)
    out = oracle_lib.grid_prune(xyz, None, None, 0.01, 0.01, 1)
    assert len(out["count"]) == 2
