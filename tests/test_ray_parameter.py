"""The clearing kernels form the ray parameter t = float32(k/K) as
float32(double(k) * RN64(1/K)) to avoid a float32 division per sample.  For
integers 1 <= k < K < 2^24 the two are equal: k/K is never a float32 rounding
boundary and lies more than 2^-49 (relative) from one, while the double
product errs by at most 2^-52.  Checked here exhaustively for K < 4096 and on
random pairs up to 2^24 (the samples' range)."""
import numpy as np


def _both(k, K):
    a = (k.astype(np.float64) * (1.0 / K.astype(np.float64))).astype(np.float32)
    b = k.astype(np.float32) / K.astype(np.float32)
    return a, b


def test_exhaustive_small_K():
    for K in range(2, 4096):
        k = np.arange(1, K, dtype=np.int64)
        a, b = _both(k, np.full_like(k, K))
        assert np.array_equal(a, b), K


def test_random_large_K():
    rng = np.random.default_rng(1)
    K = rng.integers(2, 1 << 24, 3_000_000)
    k = (rng.random(K.size) * (K - 1)).astype(np.int64) + 1
    a, b = _both(k, K)
    assert np.array_equal(a, b)
    # near the top of the range too
    K = (1 << 24) - 1 - rng.integers(0, 1000, 200_000)
    k = (rng.random(K.size) * (K - 1)).astype(np.int64) + 1
    a, b = _both(k, K)
    assert np.array_equal(a, b)
