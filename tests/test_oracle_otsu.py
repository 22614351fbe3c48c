"""The Otsu oracle (oracle/otsu.py) against the definition it restates.

* brute force: for random histograms the chosen split maximises the
  between-class variance w0 w1 (mu0 - mu1)^2 computed directly from the two
  classes' bin centres (and no earlier split reaches that maximum);
* two-level map: every split between the two levels separates them equally,
  so the first one is chosen and the mask is exactly the upper level;
* equal Gaussian modes at 0.25 and 0.75: the split falls at the midpoint
  (bin 128 +- 1);
* a constant map has no split (k* = 256, all static); NaN reads as 0.
"""
import numpy as np

from oracle import otsu as O


def _direct(hist):
    h = np.asarray(hist, np.float64)
    centres = (np.arange(O.BINS) + 0.5) / O.BINS
    N = h.sum()
    out = np.full(O.BINS, -1.0)
    for k in range(1, O.BINS):
        n0, n1 = h[:k].sum(), h[k:].sum()
        if n0 == 0 or n1 == 0:
            continue
        m0 = (h[:k] * centres[:k]).sum() / n0
        m1 = (h[k:] * centres[k:]).sum() / n1
        out[k] = (n0 / N) * (n1 / N) * (m0 - m1) ** 2
    return out


def test_split_maximises_between_class_variance():
    rng = np.random.default_rng(0)
    for trial in range(20):
        hist = rng.integers(0, 50, O.BINS) * (rng.uniform(0, 1, O.BINS) < 0.6)
        hist[rng.integers(0, O.BINS)] += 1
        hist[rng.integers(0, O.BINS)] += 1
        d = _direct(hist)
        s = O.split_scores(hist)
        if d.max() < 0:
            assert s.max() < 0
            continue
        k = int(np.argmax(s))
        assert d[k] >= d.max() * (1 - 1e-12)
        assert np.all(d[:k] < d.max() * (1 - 1e-12))
        # the scores are the variance times 512^2 N^2 wherever both classes are non-empty
        N = hist.sum()
        ok = d >= 0
        assert np.allclose(s[ok], d[ok] * (512.0 * N) ** 2, rtol=1e-9)


def test_two_levels():
    x = np.where(np.random.default_rng(1).uniform(0, 1, 5000) < 0.3, 0.8, 0.2).astype(np.float32)
    k, mask = O.otsu(x)
    assert k == int(np.floor(np.float32(0.2) * 256)) + 1
    assert np.array_equal(mask, (x > 0.5).astype(np.uint8))


def test_equal_modes_split_at_midpoint():
    rng = np.random.default_rng(2)
    x = np.concatenate([rng.normal(0.25, 0.05, 200000), rng.normal(0.75, 0.05, 200000)])
    k, _ = O.otsu(x.astype(np.float32))
    assert abs(k - 128) <= 1


def test_constant_map_and_nan():
    k, mask = O.otsu(np.full(1000, 0.4, np.float32))
    assert k == O.BINS and not mask.any()
    x = np.array([np.nan, 0.0, 1.0, 1.0], np.float32)
    assert list(O.bins_of(x)) == [0, 0, 255, 255]
