"""The oracle's isotropic, motion-aware slice (13 values per Gaussian: mean
xyz t, log s, log s_t, velocity, opacity logit, rgb), pinned to the general
rotor-form path it is a special case of.

* Zero velocity: the records, tile rectangles and counts of the rotor form
  with identity quaternions and log scales (s, s, s, s_t), bit for bit in
  FP32 (every product the rotor path adds is with an exact 0 or 1).
* Any velocity: the records of the rotor form of the same 4D covariance
  [[s^2 I + s_t^2 v v^T, s_t^2 v], [s_t^2 v^T, s_t^2]] (built by the motion
  map's eigendecomposition and quaternion factorisation, oracle/motion.py)
  through the general conditional of Eq. "4dgs", to 1e-9 in FP64.
"""
import numpy as np

import oracle
from oracle import motion
from paper_2510_01119_amd import synth


def _iso_set(n, seed, zero_velocity=False):
    rng = np.random.default_rng(seed)
    p = np.zeros((oracle.ISO_FIELDS, n))
    p[0:3] = rng.uniform(-1.0, 1.0, (3, n))
    p[3] = rng.uniform(0.0, 1.0, n)
    p[4] = rng.normal(-3.0, 0.4, n)
    p[5] = rng.normal(-1.2, 0.4, n)
    if not zero_velocity:
        p[6:9] = rng.normal(0.0, 0.5, (3, n))
    p[9] = rng.normal(0.0, 1.0, n)
    p[10:13] = rng.uniform(0.0, 1.0, (3, n))
    return p


def _rotor_base(p):
    n = p.shape[1]
    base = np.zeros((20, n))
    base[0:4] = p[0:4]
    base[4:7] = p[4]
    base[7] = p[5]
    base[8] = 1.0
    base[12] = 1.0
    base[16] = p[9]
    base[17:20] = p[10:13]
    return base


def test_zero_velocity_is_identity_rotor_bitexact():
    p = _iso_set(3000, 1, zero_velocity=True).astype(np.float32)
    for t in (0.2, 0.5, 0.9):
        view = synth.front_view(96, 64, 64.0, 3.0, t)
        a = oracle.preprocess_iso_f32(p, view)
        b = oracle.preprocess_f32(_rotor_base(p).astype(np.float32), view)
        assert a[2].sum() > 1000
        for x, y in zip(a, b):
            assert np.array_equal(x, y)


def test_velocity_matches_rotor_form_of_same_covariance():
    p = _iso_set(400, 2)
    rot = motion.init_columns(_rotor_base(p), p[5], p[6:9])
    for t in (0.1, 0.5, 0.8):
        view = synth.front_view(96, 64, 64.0, 3.0, t)
        ra, rca, ta = oracle.preprocess_iso_f64(p, view)
        rb, rcb, tb = oracle.preprocess_f64(rot, view)
        both = (ta > 0) & (tb > 0)
        assert both.sum() > 100
        assert ((ta > 0) != (tb > 0)).sum() <= 1
        d = np.abs(ra[both] - rb[both])
        scale = np.maximum(np.abs(rb[both]), 1.0)
        assert (d / scale).max() < 1e-9
