"""TEST INFRASTRUCTURE: plain numpy oracle of Otsu's threshold (Otsu, "A
threshold selection method from gray-level histograms", 1979), as used to
split a motion-probability map into static and dynamic pixels (Sec. 3.2).
Never imported by the product path.

256 uniform bins on [0, 1]: a value x (clamped, NaN as 0) falls in bin
min(255, floor(256 x)).  A split k (1..255) puts the bins below k in class
0.  With S0, S1 the count and the sum of (2i + 1) (twice the bin centre
times 256) over the bins below k and N, T their totals, the between-class
variance w0 w1 (mu0 - mu1)^2 equals A^2 / (512^2 N^2 S0 (N - S0)) with
A = T S0 - S1 N, so k* maximises A^2 / (S0 (N - S0)), evaluated in FP64 as
(A * A) / (S0 * (N - S0)); the first maximum wins.  With no split that
leaves both classes non-empty k* = 256 (everything static).
"""
import numpy as np

BINS = 256


def bins_of(prob):
    x = np.asarray(prob, np.float32)
    x = np.where(x > 0, np.where(x < 1, x, np.float32(1)), np.float32(0))  # NaN -> 0
    return np.minimum(np.floor(x * np.float32(256)).astype(np.int64), BINS - 1)


def split_scores(hist):
    """A^2 / (S0 (N - S0)) for every split k (index k; -1 where a class is
    empty, and at k = 0)."""
    h = np.asarray(hist, np.int64)
    c = 2 * np.arange(BINS, dtype=np.int64) + 1
    N, T = int(h.sum()), int((h * c).sum())
    scores = np.full(BINS, -1.0)
    s0 = s1 = 0
    for k in range(BINS):
        if k >= 1 and 0 < s0 < N:
            A = float(T * s0 - s1 * N)
            scores[k] = (A * A) / (float(s0) * float(N - s0))
        s0 += int(h[k])
        s1 += int(h[k] * c[k])
    return scores


def otsu(prob):
    """(k*, mask uint8 of prob's shape)."""
    b = bins_of(prob)
    hist = np.bincount(b.ravel(), minlength=BINS)
    s = split_scores(hist)
    k = int(np.argmax(s)) if s.max() >= 0 else BINS
    return k, (b >= k).astype(np.uint8)
