"""The stage-2 update folds each wave's largest wave speed and smallest
density into the time-step partials with 64-bit unsigned atomic max / min on
the doubles' bit patterns.  That is exact because non-negative IEEE doubles
(the speeds, after max with 0) and positive ones (the densities kept) order
like their bit patterns; NaN and negative values are excluded before the
fold.  Checked here on the host over the whole exponent range (CPU)."""
import numpy as np


def test_nonnegative_doubles_order_like_their_bits():
    rng = np.random.default_rng(7)
    for _ in range(20):
        e = rng.uniform(-1074, 1023, size=4096)
        x = np.ldexp(rng.uniform(1.0, 2.0, size=4096), np.floor(e).astype(int))
        x[rng.integers(0, 4096, size=64)] = 0.0
        x[:8] = [0.0, 5e-324, 2.2250738585072014e-308, 1.0, 1e300, np.finfo(float).max, 1e-300, 3.0]
        bits = x.view(np.uint64)
        assert np.argsort(bits, kind="stable").tolist() == np.argsort(x, kind="stable").tolist()
        assert x[np.argmax(bits)] == x.max() and x[np.argmin(bits)] == x.min()


def test_fold_initial_values():
    """The emptied partials (speed 0, density 1e300) are neutral for max and
    min over the values the fold admits."""
    s0, r0 = np.float64(0.0).view(np.uint64), np.float64(1e300).view(np.uint64)
    for v in (5e-324, 1e-12, 1.0, 3.7e2, 1e299):
        b = np.float64(v).view(np.uint64)
        assert max(s0, b) == b and min(r0, b) == b
