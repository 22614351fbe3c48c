"""Pins for the oracle's project-written FP32 exp and ln (Cody-Waite exp,
atanh-series ln): against the C library's double-precision routines."""
import numpy as np
import pytest


def _ulp_err(got, ref):
    ref32 = np.float32(ref)
    ulp = np.spacing(np.abs(ref32)).astype(np.float64)
    return abs(float(got) - ref) / ulp


def test_expf_matches_libm(oracle_lib):
    rng = np.random.default_rng(0)
    xs = np.concatenate([rng.uniform(-87, 88, 4000), rng.uniform(-1, 1, 2000),
                         [0.0, 1.0, -1.0, -86.99, 87.99, 1e-8, -1e-8]]).astype(np.float32)
    worst = 0.0
    for x in xs:
        worst = max(worst, _ulp_err(oracle_lib.expf(x), np.exp(np.float64(x))))
    assert worst <= 2.0, worst


def test_expf_special(oracle_lib):
    assert oracle_lib.expf(0.0) == 1.0
    assert oracle_lib.expf(-100.0) == 0.0
    assert oracle_lib.expf(100.0) == float("inf")
    assert np.isnan(oracle_lib.expf(float("nan")))


def test_logf_matches_libm(oracle_lib):
    rng = np.random.default_rng(1)
    xs = np.concatenate([np.exp(rng.uniform(-80, 80, 4000)), rng.uniform(0.5, 2.0, 2000),
                         [1.0, 2.0, 255.0, 0.70710677, 1.4142135]]).astype(np.float32)
    worst = 0.0
    for x in xs:
        ref = np.log(np.float64(x))
        if ref == 0.0:
            assert oracle_lib.logf(x) == 0.0
            continue
        worst = max(worst, _ulp_err(oracle_lib.logf(x), ref))
    # near x = 1 the rounding of u = (m-1)/(m+1) dominates: a few ulp
    assert worst <= 3.0, worst


def test_logf_special(oracle_lib):
    assert oracle_lib.logf(1.0) == 0.0
    assert oracle_lib.logf(0.0) == float("-inf")
    assert np.isnan(oracle_lib.logf(-1.0))
