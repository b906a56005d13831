"""Pins of the parabolic short-characteristics oracle (the higher-order
source interpolant mentioned with Eq. 4-7): the three coefficients integrate
any quadratic source exactly over a layer (checked against scipy's
quadrature), a whole sweep is exact for a source quadratic in optical depth,
a linear source gives the linear scheme's result, an isothermal column gives
pi B, and on a smooth curved source the parabolic sweep converges at third
order where the linear one converges at second."""
import numpy as np
import pytest
from scipy import integrate

import oracle


@pytest.mark.parametrize("du,dd", [(1e-9, 3e-9), (2e-6, 1e-6), (1e-3, 2e-3), (0.05, 0.01),
                                   (0.3, 0.7), (1.0, 1.0), (2.5, 0.4), (12.0, 30.0), (45.0, 5.0)])
def test_coefficients_integrate_quadratics(du, dd):
    a, b, g = oracle.sc_para_coeffs(du, dd)
    assert abs((a + b + g) - (-np.expm1(-du))) < 1e-14
    rng = np.random.default_rng(int(du * 1000 + dd * 10))
    for _ in range(3):
        c0, c1, c2 = rng.uniform(-1, 1, 3)
        S = lambda x: c0 + c1 * x + c2 * x * x
        want, _ = integrate.quad(lambda x: S(x) * np.exp(-x), 0.0, du, epsabs=0, epsrel=1e-13)
        got = a * S(-dd) + b * S(0.0) + g * S(du)
        assert abs(got - want) <= 1e-12 * abs(want)


def test_moments_of_thin_layers_match_the_incomplete_gamma_function():
    """The coefficients rest on w_n = gamma(n+1, du); scipy's regularised
    incomplete gamma gives them independently, down to du = 1e-12."""
    from scipy import special
    for du in (1e-12, 1e-8, 1e-4, 0.2, 3.0, 29.5, 30.5, 60.0):
        dd = 0.7 * du
        w0, w1, w2 = -np.expm1(-du), special.gammainc(2, du), 2.0 * special.gammainc(3, du)
        a, b, g = oracle.sc_para_coeffs(du, dd)
        assert abs(g - (w2 + dd * w1) / (du * (du + dd))) <= 1e-13 * abs(g)
        assert abs(a - (w2 - du * w1) / (dd * (du + dd))) <= 1e-12 * abs(a)
        assert abs((a + b + g) - w0) <= 1e-13 * w0


def _tau_grid(n, top_thin=1e-10, tot=6.0, seed=3):
    rng = np.random.default_rng(seed)
    dtau = rng.uniform(0.5, 1.5, n - 1)
    dtau *= tot / dtau.sum()
    dtau[-1] = top_thin
    tau = np.concatenate([np.cumsum(dtau[::-1])[::-1], [0.0]])   # tau at levels, bottom first
    return dtau, tau


@pytest.mark.parametrize("mu", [0.15, 0.5, 1.0])
def test_sweep_is_exact_for_a_quadratic_source(mu):
    """Eq. 1 with the source quadratic in tau below the top layer and linear
    across the top layer (the step with no downwind level), integrated by
    quadrature: the parabolic sweep reproduces it."""
    dtau, tau = _tau_grid(25, top_thin=0.3)
    S_of = lambda t: 2.0 + 0.7 * t - 0.09 * t * t
    S = S_of(tau)
    t1 = tau[-2]
    S_eff = lambda t: S_of(t) if t >= t1 else S[-1] + (S[-2] - S[-1]) * t / t1
    got = oracle.sc_intensity_para(dtau, S, mu)
    integ = 0.0
    for lo, hi in zip(tau[1:], tau[:-1]):
        v, _ = integrate.quad(lambda t: S_eff(t) * np.exp(-t / mu) / mu, lo, hi, epsabs=0,
                              epsrel=1e-13, limit=200)
        integ += v
    want = integ + S[0] * np.exp(-tau[0] / mu)
    assert abs(got - want) < 1e-12 * abs(want)
    # the linear scheme is not exact here
    assert abs(oracle.sc_intensity(dtau, S, mu) - want) > 1e-6 * abs(want)


def test_linear_source_and_isothermal_reduce_to_the_linear_scheme():
    dtau, tau = _tau_grid(30, top_thin=0.2)
    S = 1.0 + 0.4 * tau
    for mu in (0.2, 0.7):
        assert abs(oracle.sc_intensity_para(dtau, S, mu) - oracle.sc_intensity(dtau, S, mu)) < 1e-13
    Sc = np.full(30, 3.25)
    assert abs(oracle.sc_intensity_para(dtau, Sc, 0.4) - 3.25) < 1e-13
    assert abs(oracle.sc_flux(dtau, Sc, 3, order=2) - np.pi * 3.25) < 1e-12


def test_zero_optical_depth_layers():
    """A transparent layer adds nothing, and the step below it falls back to the
    linear coefficients (no division by its zero path length)."""
    dtau = np.array([0.8, 0.0, 0.5, 0.0])
    S = np.array([3.0, 2.0, 1.5, 1.2, 1.1])
    I = oracle.sc_intensity_para(dtau, S, 0.6)
    # by hand: step 0 linear (downwind layer empty), step 1 nothing, step 2 linear (downwind empty)
    def lin(I, d, S1, S0):
        e = np.exp(-d)
        u = -np.expm1(-d) / d
        return e * I + (1 - u) * S1 + (u - e) * S0
    want = lin(lin(3.0, 0.8 / 0.6, 2.0, 3.0), 0.5 / 0.6, 1.2, 1.5)
    assert abs(I - want) < 1e-14


def test_third_order_convergence_on_a_curved_source():
    """S = exp(-t/2) + 0.3 sin(t): halving the layers cuts the parabolic error
    by about 8 (third order) and the linear one by about 4."""
    mu = 0.6
    S_of = lambda t: np.exp(-t / 2) + 0.3 * np.sin(t) + 1.0
    integ, _ = integrate.quad(lambda t: S_of(t) * np.exp(-t / mu) / mu, 0.0, 8.0, epsabs=0,
                              epsrel=1e-13, limit=400)
    want = integ + S_of(8.0) * np.exp(-8.0 / mu)
    errs = {}
    for n in (80, 160, 320):
        tau = np.linspace(8.0, 0.0, n + 1)
        dtau = -np.diff(tau)
        S = S_of(tau)
        errs[n] = (abs(oracle.sc_intensity(dtau, S, mu) - want),
                   abs(oracle.sc_intensity_para(dtau, S, mu) - want))
    r_lin = errs[160][0] / errs[320][0]
    r_par = errs[160][1] / errs[320][1]
    assert 3.5 < r_lin < 4.5
    assert r_par > 6.5
    assert errs[320][1] < 0.2 * errs[320][0]
