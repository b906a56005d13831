"""The closed form the FP32 observation layouts use for the Gaussian
normalisation sums Z = sum_{k=a}^{b} exp(-k^2 / (2 s^2)) (a <= 0 <= b):
the Euler-Maclaurin formula with the integral (erf) and the endpoint terms of
f, f', f''' and f^(5).  Checked here, in FP64 numpy, against the direct sums
for the bounds the kernel relies on (relative error below 1e-9 for s >= 4,
below 5e-12 for s >= 8); the GPU parity tests check the kernel against the
oracle's direct sums."""
import numpy as np
from scipy.special import erf


def direct(s, a, b):
    k = np.arange(a, b + 1, dtype=np.float64)
    return float(np.sum(np.exp(-k * k / (2.0 * s * s))))


def euler_maclaurin(s, a, b):
    f = lambda x: np.exp(-x * x / (2.0 * s * s))
    d1 = lambda x: -(x / s**2) * f(x)
    d3 = lambda x: (3.0 * x / s**4 - x**3 / s**6) * f(x)
    d5 = lambda x: (-15.0 * x / s**6 + 10.0 * x**3 / s**8 - x**5 / s**10) * f(x)
    r = 1.0 / (s * np.sqrt(2.0))
    return (s * np.sqrt(np.pi / 2.0) * (erf(b * r) - erf(a * r)) + 0.5 * (f(a) + f(b))
            + (d1(b) - d1(a)) / 12.0 - (d3(b) - d3(a)) / 720.0 + (d5(b) - d5(a)) / 30240.0)


def cases(s):
    h = int(np.floor(5.0 * s))
    # whole cut, and cuts shortened by either end of the window
    short = [(a, b) for a in range(-6, 1) for b in range(0, 7)]
    return [(-h, h), (0, h), (-h, 0), (-h, h // 3), (-(h // 2), h), (-3, h), (-h, 7)] + short


def test_error_bounds_against_direct_sums():
    rng = np.random.default_rng(0)
    s_values = np.concatenate([np.linspace(4.0, 8.0, 33),
                               np.exp(rng.uniform(np.log(8.0), np.log(4000.0), 120))])
    for s in s_values:
        for a, b in cases(s):
            d = direct(s, a, b)
            e = abs(euler_maclaurin(s, a, b) - d) / d
            assert e < (1e-9 if s < 8.0 else 5e-12), (s, a, b, e)


def test_single_tap_and_symmetry():
    for s in (4.0, 37.5, 900.0):
        assert abs(euler_maclaurin(s, 0, 0) - 1.0) < 1e-15
        h = int(5 * s)
        assert abs(euler_maclaurin(s, -h, 3) - euler_maclaurin(s, -3, h)) < 1e-12 * direct(s, -h, 3)


def test_below_the_threshold_the_formula_would_not_do():
    # why the kernel sums directly below s = 4: the truncated series drifts
    worst = max(abs(euler_maclaurin(s, a, b) - direct(s, a, b)) / direct(s, a, b)
                for s in np.linspace(1.0, 2.0, 11) for a, b in cases(s))
    assert worst > 1e-8
