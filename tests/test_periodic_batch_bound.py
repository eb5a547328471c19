"""The bound behind the periodic passes' per-batch shortcut: FP32 subtraction
is monotonic (round to nearest even), so for x_i inside [lo, hi] the computed
difference fl(x_j - x_i) lies between fl(x_j - hi) and fl(x_j - lo). When both
of those are at most half a period in magnitude, no pair of the batch needs a
minimum image and the tiles may skip the test with the same results."""
import numpy as np


def test_fp32_difference_is_bounded_by_the_box_ends():
    rng = np.random.default_rng(2024)
    f = np.float32
    for scale in (1.0, 1e-3, 1e3):
        lo = (rng.random(200000) * scale).astype(f)
        hi = (lo + rng.random(200000).astype(f) * f(0.1 * scale)).astype(f)
        xi = (lo + (hi - lo) * rng.random(200000).astype(f)).astype(f)
        xi = np.clip(xi, lo, hi)
        xj = (rng.random(200000) * 2 * scale - 0.5 * scale).astype(f)
        d = np.abs(xj - xi)
        bound = np.maximum(np.abs(xj - lo), np.abs(xj - hi))
        assert d.dtype == np.float32 and bound.dtype == np.float32
        assert np.all(d <= bound)


def test_bound_holds_at_the_box_ends_and_ties():
    f = np.float32
    lo, hi = f(0.25), f(np.nextafter(f(0.25), f(1)))
    for xj in (f(0.75), f(0.75) + f(1e-8), f(-0.25), lo, hi):
        for xi in (lo, hi):
            assert abs(f(xj - xi)) <= max(abs(f(xj - lo)), abs(f(xj - hi)))
