"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test states the property it pins and the passage it follows.  None of
them re-types the oracle's own formula as the expected value: they use
closed forms of special cases (isothermal, transparent, opaque columns; a
source linear in optical depth), brute-force quadrature of the formal
solution (Eq. 1) and of the Schwarzschild-Milne flux (Eq. 3), library
routines (numpy's Gauss-Legendre, scipy's exponential integrals and physical
constants), and exactness properties of the interpolation, convolution and
binning.
"""
import numpy as np
import pytest
from scipy import constants as sc
from scipy import integrate, special

import oracle
import workloads as wl

# independent cgs constants (scipy's CODATA values, converted from SI)
H = sc.h * 1e7
C = sc.c * 1e2
KB = sc.k * 1e7
SIGMA_SB = sc.Stefan_Boltzmann * 1e3
AMU = sc.physical_constants["atomic mass constant"][0] * 1e3
# h, c and k_B are exact since the 2019 SI; m_u is not, and scipy may carry a
# later CODATA adjustment than the 2018 value used by the forward model
# (1.66053906660e-24 g), so checks through m_u allow for that revision.
AMU_RTOL = 5e-9


def planck_ref(nu, T):
    x = H * C * nu / (KB * T)
    return 2 * H * C * C * nu ** 3 / np.expm1(x)


@pytest.fixture(scope="module")
def c1():
    return wl.c1_table()


# ------------------------------------------------------------------ Eq. 8


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 8, 16, 48])
def test_p8_gauss_nodes_match_library(n):
    """P8: half-range Gauss-Legendre nodes equal numpy's rule mapped to [0, 1]."""
    mu, w = oracle.gauss_legendre01(n)
    t, wt = np.polynomial.legendre.leggauss(n)
    np.testing.assert_allclose(mu, 0.5 * (1 + t), rtol=0, atol=2e-15)
    np.testing.assert_allclose(w, 0.5 * wt, rtol=2e-14 if n <= 16 else 5e-12, atol=0)
    assert abs(w.sum() - 1) < 1e-14
    assert abs((w * mu).sum() - 0.5) < 1e-14      # exact flux of an isotropic field
    if n >= 2:
        assert abs((w * mu * mu).sum() - 1.0 / 3.0) < 1e-14


def test_p8_closed_form_two_and_three_point():
    mu, w = oracle.gauss_legendre01(2)
    np.testing.assert_allclose(mu, [0.5 - 0.5 / np.sqrt(3), 0.5 + 0.5 / np.sqrt(3)], atol=1e-15)
    np.testing.assert_allclose(w, [0.5, 0.5], atol=1e-15)
    mu, w = oracle.gauss_legendre01(3)
    np.testing.assert_allclose(mu, [0.5 - 0.5 * np.sqrt(0.6), 0.5, 0.5 + 0.5 * np.sqrt(0.6)],
                               atol=1e-15)
    np.testing.assert_allclose(w, [5 / 18, 8 / 18, 5 / 18], atol=1e-15)


# ------------------------------------------------------------------ Eq. 2


@pytest.mark.parametrize("T", [50.0, 300.0, 1000.0, 3000.0])
def test_p9_planck_integrates_to_stefan_boltzmann(T):
    """P9: pi int B_nu dnu = sigma_SB T^4 (Planck's law in wavenumber form)."""
    numax = 60.0 * KB * T / (H * C)
    edges = np.linspace(0.0, numax, 61)
    tot = 0.0
    for a, b in zip(edges[:-1], edges[1:]):
        a = max(a, 1e-9 * numax)
        val, _ = integrate.quad(lambda v: oracle.planck(v, T)[()], a, b, epsabs=0, epsrel=1e-13,
                                limit=200)
        tot += val
    assert abs(np.pi * tot / (SIGMA_SB * T ** 4) - 1) < 1e-8


def test_p9_planck_limits():
    T = 1000.0
    # Wien: x >> 1
    nu = 200.0 * KB * T / (H * C)
    wien = 2 * H * C * C * nu ** 3 * np.exp(-H * C * nu / (KB * T))
    assert abs(oracle.planck(nu, T)[()] / wien - 1) < 1e-12
    # Rayleigh-Jeans with its first corrections: x << 1
    nu = 1e-4 * KB * T / (H * C)
    x = H * C * nu / (KB * T)
    rj = 2 * C * KB * T * nu * nu * (1 - x / 2 + x * x / 12)
    assert abs(oracle.planck(nu, T)[()] / rj - 1) < 1e-12
    np.testing.assert_allclose(oracle.planck([500.0, 5000.0], [700.0, 2500.0]),
                               planck_ref(np.array([500.0, 5000.0]), np.array([700.0, 2500.0])),
                               rtol=1e-13)


# ------------------------------------------------------------- Eq. 4-7


def test_p6_linear_source_is_reproduced_exactly():
    """P6: with S = a + b tau (tau measured from the top) the linear-source
    scheme is exact for any layer partition: I(0, mu) = a + b mu (1 - e^{-T/mu})
    (formal solution with the semi-infinite continuation S = S(T) below)."""
    rng = np.random.default_rng(7)
    for L in (2, 3, 7, 40):
        dtau = 10.0 ** rng.uniform(-6, 1.5, L - 1)
        tau = np.concatenate([np.cumsum(dtau[::-1])[::-1], [0.0]])   # tau at levels
        a, b = rng.uniform(0.5, 2.0), rng.uniform(-0.3, 3.0)
        S = a + b * tau
        for mu in (0.05, 0.3, 0.7, 1.0):
            got = oracle.sc_intensity(dtau, S, mu)
            want = a + b * mu * (1 - np.exp(-tau[0] / mu))
            assert abs(got / want - 1) < 1e-12, (L, mu, got, want)


def _formal_solution(dtau, S, mu):
    """Eq. 1 at the top, S piecewise linear in tau, constant S_0 below the bottom."""
    tau = np.concatenate([np.cumsum(dtau[::-1])[::-1], [0.0]])

    def s_of_t(t):
        return np.interp(t, tau[::-1], S[::-1])

    tot = 0.0
    for l in range(len(dtau)):
        lo, hi = tau[l + 1], tau[l]
        v, _ = integrate.quad(lambda t: s_of_t(t) * np.exp(-t / mu) / mu, lo, hi, epsabs=0,
                              epsrel=1e-13, limit=200)
        tot += v
    return tot + S[0] * np.exp(-tau[0] / mu)


def test_p7_brute_force_formal_solution():
    """P7: the recurrence equals Eq. 1 integrated by quadrature on 2-4 layers."""
    rng = np.random.default_rng(11)
    for L in (2, 3, 4, 5):
        for _ in range(4):
            dtau = 10.0 ** rng.uniform(-3, 1, L - 1)
            S = rng.uniform(0.1, 5.0, L)
            for mu in (0.1, 0.5, 0.9):
                got = oracle.sc_intensity(dtau, S, mu)
                want = _formal_solution(dtau, S, mu)
                assert abs(got / want - 1) < 1e-11, (L, mu)


def test_p7_flux_converges_to_schwarzschild_milne():
    """P7: with many angles, Eq. 8 tends to Eq. 3, F = 2 pi int S E_2(t) dt
    (+ 2 pi S_0 E_3(T) from the semi-infinite continuation)."""
    rng = np.random.default_rng(13)
    dtau = 10.0 ** rng.uniform(-2, 0.5, 4)
    S = rng.uniform(0.5, 3.0, 5)
    tau = np.concatenate([np.cumsum(dtau[::-1])[::-1], [0.0]])

    def s_of_t(t):
        return np.interp(t, tau[::-1], S[::-1])

    tot = 0.0
    for l in range(4):
        v, _ = integrate.quad(lambda t: s_of_t(t) * special.expn(2, t), tau[l + 1], tau[l],
                              epsabs=0, epsrel=1e-12, limit=400)
        tot += v
    milne = 2 * np.pi * (tot + S[0] * special.expn(3, tau[0]))
    err = [abs(oracle.sc_flux(dtau, S, n) / milne - 1) for n in (4, 16, 64)]
    assert err[2] < 1e-6 and err[2] <= err[0]


def test_p14_closed_form_scan_equals_recurrence():
    """P14: I_top = S_0 e^{-tau_0/mu} + sum_l e^{-tau_{l+1}/mu} (beta_l S_{l+1} + gamma_l S_l)
    with the transmission written through cumulative optical depth."""
    rng = np.random.default_rng(17)
    L = 30
    dtau = 10.0 ** rng.uniform(-5, 0.5, L - 1)
    S = rng.uniform(0.1, 3.0, L)
    tau = np.concatenate([np.cumsum(dtau[::-1])[::-1], [0.0]])
    for mu in (0.2, 0.8):
        d = dtau / mu
        # coefficients from the definition of the linear-source integral:
        # beta = int_0^1 s e^{-d(1-s)} d ds ... written as series-free closed forms
        e = np.exp(-d)
        beta = 1 - (1 - e) / d
        gamma = (1 - e) / d - e
        scan = S[0] * np.exp(-tau[0] / mu) + np.sum(np.exp(-tau[1:] / mu) *
                                                     (beta * S[1:] + gamma * S[:-1]))
        got = oracle.sc_intensity(dtau, S, mu)
        assert abs(got / scan - 1) < 1e-12


def test_linear_source_coefficients_are_the_layer_integrals():
    """The coefficients are the weights of S_{l+1}, S_l in int_0^D S(t) e^{-t} dt
    for S linear between the two levels (the upwind point is the deeper level):
    check by quadrature with S_l = 0, S_{l+1} = 1 and vice versa."""
    for D in (1e-3, 0.1, 1.0, 7.0):
        # one layer, S = [S_bottom, S_top]; intensity with I_bottom = 0 is
        # obtained as I(S) - e^{-D} S_bottom
        w_top = oracle.sc_intensity([D], [0.0, 1.0], 1.0)
        w_bot = oracle.sc_intensity([D], [1.0, 0.0], 1.0) - np.exp(-D)
        # t measured from the top of the layer down to D
        q_top, _ = integrate.quad(lambda t: (1 - t / D) * np.exp(-t), 0, D, epsabs=0, epsrel=1e-13)
        q_bot, _ = integrate.quad(lambda t: (t / D) * np.exp(-t), 0, D, epsabs=0, epsrel=1e-13)
        assert abs(w_top / q_top - 1) < 1e-10
        assert abs(w_bot / q_bot - 1) < 1e-10


# ------------------------------------------------------ isothermal / limits


def _isothermal_column(T, L=21, x=1e-3, log_g=4.75):
    p = wl.levels(L, 2.0, -4.0)
    return wl.Column(p, np.full(L, T), np.array([x]), log_g, wl.scale_factor(1.0))


@pytest.mark.parametrize("T", [900.0, 1000.0, 412.5])
@pytest.mark.parametrize("n_mu", [1, 2, 3, 5])
def test_p3_isothermal_column_emits_pi_b(c1, T, n_mu):
    """P3: an isothermal column emits F+ = pi B(T) whatever its opacity (Eq. 1-8)."""
    col = _isothermal_column(T)
    w = wl.Window(0, c1.n_nu, 1)
    sub = np.arange(0, c1.n_nu, 7)
    fp = oracle.fplus(c1, col, w, n_mu, sub)
    want = np.pi * planck_ref(c1.nu0_cm + sub * c1.dnu_cm, T)
    np.testing.assert_allclose(fp, want, rtol=2e-13)


def test_p3_full_chain_delta_profile(c1):
    """P3 through stages 3: with a delta instrument profile, each bin is the
    trapezoid mean of pi B times f (R/d)^2 (Eq. 9, 17, binning)."""
    col = _isothermal_column(1000.0)
    obs = wl.c1_obs(c1)
    res = oracle.forward(c1, col, obs.window, 1e12, obs.edges_cm, 3)
    nu = c1.nu(0, c1.n_nu, 1)
    fb = np.pi * planck_ref(nu, 1000.0)
    idx = res["edge_idx"]
    want = []
    for a, b in zip(idx[:-1], idx[1:]):
        seg = fb[a:b + 1]
        want.append(np.trapezoid(seg, nu[a:b + 1]) / (nu[b] - nu[a]))
    np.testing.assert_allclose(res["bins"], col.scale * np.array(want), rtol=1e-13)


def test_p4_opaque_isothermal_top_layer():
    """P4: an isothermal top layer with dtau >= 60 screens everything below."""
    rng = np.random.default_rng(3)
    L, n = 12, 5
    T = rng.uniform(400, 2000, L)
    T[-2] = T[-1] = 800.0
    nu = np.linspace(1000, 9000, n)
    dz = np.ones(L - 1)
    chi = 10.0 ** rng.uniform(-3, 0, (L, n))
    chi[-2:, :] = 60.0
    fp = oracle.rt_emission(chi, dz, T, nu, 3)
    np.testing.assert_allclose(fp, np.pi * planck_ref(nu, 800.0), rtol=1e-12)


def test_p5_transparent_column_transmits_the_boundary():
    """P5: chi = 0 everywhere gives F+ = pi B(T_bottom) (boundary reading)."""
    rng = np.random.default_rng(5)
    L, n = 9, 4
    T = rng.uniform(300, 2500, L)
    nu = np.linspace(500, 8000, n)
    fp = oracle.rt_emission(np.zeros((L, n)), np.ones(L - 1), T, nu, 3)
    np.testing.assert_allclose(fp, np.pi * planck_ref(nu, T[0]), rtol=1e-15)


# ------------------------------------------------------------ Sect. 2.3


def _bilinear_table(rng, S=2, nT=4, nP=5, n_nu=6):
    T = np.sort(rng.uniform(100, 3000, nT))
    lp = np.sort(rng.uniform(-6, 3, nP))
    a = rng.uniform(-28, -20, (S, 1, 1, n_nu))
    b = rng.uniform(-1e-3, 1e-3, (S, 1, 1, n_nu))
    c = rng.uniform(-0.5, 0.5, (S, 1, 1, n_nu))
    d = rng.uniform(-2e-4, 2e-4, (S, 1, 1, n_nu))
    TT = T[None, :, None, None]
    PP = lp[None, None, :, None]
    tab = a + b * TT + c * PP + d * TT * PP
    coef = (a[:, 0, 0], b[:, 0, 0], c[:, 0, 0], d[:, 0, 0])
    table = wl.Table(T_K=T, log10_p_bar=lp, nu0_cm=1000.0, dnu_cm=1.0, n_nu=n_nu,
                     log10_sigma=np.ascontiguousarray(tab), molar_mass=np.full(S, 20.0),
                     log10_k_cia=None)
    return table, coef


def test_p2_bilinear_reproduces_bilinear_functions():
    """P2: bilinear interpolation on log sigma is exact for a + bT + c lp + d T lp."""
    rng = np.random.default_rng(19)
    table, (a, b, c, d) = _bilinear_table(rng)
    S = table.n_species
    L = 6
    T = rng.uniform(table.T_K[0], table.T_K[-1], L)
    lp = np.sort(rng.uniform(table.log10_p_bar[0], table.log10_p_bar[-1], L))[::-1]
    x = np.array([1e-3, 3e-4])
    col = wl.Column(10.0 ** lp, T, x, 4.0, 1.0)
    chi_each = []
    for s in range(S):
        xs = np.zeros(S)
        xs[s] = x[s]
        chi_each.append(oracle.opacity(table, wl.Column(col.p_bar, T, xs, 4.0, 1.0),
                                       np.arange(table.n_nu)))
    n_tot = col.p_bar * 1e6 / (KB * T)
    for s in range(S):
        want = x[s] * n_tot[:, None] * 10.0 ** (a[s] + b[s] * T[:, None] + c[s] * np.log10(
            col.p_bar)[:, None] + d[s] * T[:, None] * np.log10(col.p_bar)[:, None])
        np.testing.assert_allclose(chi_each[s], want, rtol=1e-12)
    np.testing.assert_allclose(oracle.opacity(table, col, np.arange(table.n_nu)),
                               chi_each[0] + chi_each[1], rtol=1e-14)


def test_p1_nodes_are_exact_and_outside_clamps(c1):
    """P1: a level on a table node returns that node's value; outside the table
    the lookup clamps to the edge (no extrapolation)."""
    lp = np.array([2.0, 0.5, -1.0, -2.5, -4.0])
    T = np.array([1500.0, 1200.0, 900.0, 600.0, 300.0])
    col = wl.Column(10.0 ** lp, T, np.array([1e-3]), 4.75, 1.0)
    nu_idx = np.arange(0, c1.n_nu, 13)
    chi = oracle.opacity(c1, col, nu_idx)
    n = col.x[0] * col.p_bar * 1e6 / (KB * T)
    for l in range(5):
        it = 4 - l
        ip = 4 - l
        want = n[l] * 10.0 ** c1.log10_sigma[0, it, ip, nu_idx]
        np.testing.assert_allclose(chi[l], want, rtol=5e-14)
    # clamping: T below / above the axis, p above / below it
    col2 = wl.Column(10.0 ** np.array([3.0, -5.0]), np.array([5000.0, 100.0]), np.array([1e-3]),
                     4.75, 1.0)
    chi2 = oracle.opacity(c1, col2, nu_idx)
    n2 = 1e-3 * col2.p_bar * 1e6 / (KB * col2.T_K)
    np.testing.assert_allclose(chi2[0], n2[0] * 10.0 ** c1.log10_sigma[0, 4, 4, nu_idx], rtol=5e-14)
    np.testing.assert_allclose(chi2[1], n2[1] * 10.0 ** c1.log10_sigma[0, 0, 0, nu_idx], rtol=5e-14)


def test_cia_binary_absorption_closed_form():
    """CIA: chi = n_H2^2 k_HH + n_H2 n_He k_HHe, linear in T on log k (Sect. 2.3).
    Filler-only gas (x_s = 0), log k linear in T, distinct pairs."""
    rng = np.random.default_rng(23)
    T_ax = np.array([200.0, 800.0, 1500.0, 2500.0])
    n_nu = 5
    a = rng.uniform(-47, -45, (2, 1, n_nu))
    b = rng.uniform(-1e-4, 1e-4, (2, 1, n_nu))
    cia = a + b * T_ax[None, :, None]
    table = wl.Table(T_K=T_ax, log10_p_bar=np.array([-3.0, 2.0]), nu0_cm=2000.0, dnu_cm=2.0,
                     n_nu=n_nu, log10_sigma=np.full((1, 4, 2, n_nu), -30.0),
                     molar_mass=np.array([18.0]), log10_k_cia=np.ascontiguousarray(cia))
    T = np.array([1800.0, 950.0, 333.0])
    p = np.array([10.0, 1.0, 0.1])
    col = wl.Column(p, T, np.array([0.0]), 4.5, 1.0)
    chi = oracle.opacity(table, col, np.arange(n_nu))
    n = p * 1e6 / (KB * T)
    xh2 = 1.0 / (1.0 + table.he_h2_ratio)
    xhe = table.he_h2_ratio * xh2
    kh = 10.0 ** (a[0] + b[0] * T[:, None])
    khe = 10.0 ** (a[1] + b[1] * T[:, None])
    want = (xh2 * n[:, None]) ** 2 * kh + (xh2 * n[:, None]) * (xhe * n[:, None]) * khe
    # plus the (negligible but present) species floor with x = 0 contributes 0
    np.testing.assert_allclose(chi, want, rtol=1e-13)


def test_p10_isothermal_constant_table_optical_depth():
    """P10: isothermal, constant sigma: dz = H ln(p_l / p_l+1) with the pressure
    scale height H = k_B T / (mubar m_u g), and
    dtau = x sigma / (mubar m_u g) (p_l + p_l+1)/2 ln(p_l / p_l+1) -- T-free; the
    column optical depth approaches the hydrostatic x sigma (p_0 - p_top)/(mubar m_u g)."""
    n_nu = 3
    sigma = 1e-22
    table = wl.Table(T_K=np.array([100.0, 4000.0]), log10_p_bar=np.array([-7.0, 4.0]),
                     nu0_cm=1000.0, dnu_cm=1.0, n_nu=n_nu,
                     log10_sigma=np.full((1, 2, 2, n_nu), np.log10(sigma)),
                     molar_mass=np.array([18.015]), log10_k_cia=None)
    L = 201
    p = wl.levels(L, 2.0, -4.0)
    x = 2e-3
    g = 10.0 ** 4.3
    for T in (700.0, 1900.0):
        col = wl.Column(p, np.full(L, T), np.array([x]), 4.3, 1.0)
        st = oracle.column_state(table, col)
        xh2 = (1 - x) / 1.17
        mubar = x * 18.015 + xh2 * 2.016 + 0.17 * xh2 * 4.0026
        assert abs(st["mubar"] / mubar - 1) < 1e-15
        Hs = KB * T / (mubar * AMU * g)
        np.testing.assert_allclose(st["dz"], Hs * np.log(p[:-1] / p[1:]), rtol=AMU_RTOL)
        chi = oracle.opacity(table, col, np.arange(n_nu))
        dtau = 0.5 * (chi[:-1, 0] + chi[1:, 0]) * st["dz"]
        pd = p * 1e6
        want = x * sigma / (mubar * AMU * g) * 0.5 * (pd[:-1] + pd[1:]) * np.log(p[:-1] / p[1:])
        np.testing.assert_allclose(dtau, want, rtol=AMU_RTOL)
        hydro = x * sigma * (pd[0] - pd[-1]) / (mubar * AMU * g)
        assert abs(dtau.sum() / hydro - 1) < 1e-3


def _planck_inverse(nu, S):
    """The temperature whose Planck intensity at wavenumber nu is S."""
    return H * C * nu / (KB * np.log1p(2 * H * C * C * nu ** 3 / S))


@pytest.mark.parametrize("n_mu", [1, 2, 3, 5])
def test_layer_optical_depth_is_the_integral_of_a_linear_opacity(n_mu):
    """Sect. 2.8 ("calculation of the optical depths"), reading: a layer's
    optical depth is the integral of chi over its geometric thickness with chi
    varying linearly between the two levels.  Pin: take chi exactly linear in
    height, chi(z) = c0 + c1 z, so the optical depth above height z is the
    closed form c0 (Z - z) + c1 (Z^2 - z^2) / 2 (Z: the top), and choose the
    level temperatures by inverting Planck's law so that S = B_nu(T) is exactly
    linear in that optical depth, S = a + b tau.  The linear-source scheme is
    exact for such a source (Eq. 4-7), so the oracle's RT entry, which forms
    every layer's optical depth from chi at the levels and the thicknesses
    itself, must return the closed-form flux of Eq. 8 with Eq. 1:
    F+ = 2 pi sum_k w_k mu_k (a + b mu_k (1 - exp(-tau_0 / mu_k))).
    Chi is steep across every layer (it falls by a factor 1.5-6 over the
    column), so a rectangle rule, a missing half or the wrong level would move
    both the optical depths at the levels and the total."""
    rng = np.random.default_rng(41 + n_mu)
    t, wt = np.polynomial.legendre.leggauss(n_mu)
    mu, w = 0.5 * (t + 1.0), 0.5 * wt
    nu = 2300.0
    for L in (2, 3, 6, 25, 80):
        for _ in range(4):
            dz = 10.0 ** rng.uniform(5.0, 7.0, L - 1)       # cm, bottom layer first
            z = np.concatenate([[0.0], np.cumsum(dz)])      # level heights
            Z = z[-1]
            tau_tot = 10.0 ** rng.uniform(-0.5, 0.9)
            grad = rng.uniform(0.5, 5.0)
            kappa = tau_tot / (Z * (1.0 + grad / 2.0))
            c0, c1 = kappa * (1.0 + grad), -kappa * grad / Z
            chi = c0 + c1 * z
            tau = c0 * (Z - z) + c1 * (Z * Z - z * z) / 2.0
            assert abs(tau[0] / tau_tot - 1) < 1e-12 and tau[-1] == 0.0
            S_top, S_bot = planck_ref(nu, rng.uniform(500.0, 900.0)), planck_ref(nu, 2200.0)
            a, b = S_top, (S_bot - S_top) / tau[0]
            T = _planck_inverse(nu, a + b * tau)
            got = oracle.rt_emission(chi[:, None], dz, T, np.array([nu]), n_mu)[0]
            want = 2 * np.pi * np.sum(w * mu * (a + b * mu * (1.0 - np.exp(-tau[0] / mu))))
            assert abs(got / want - 1) < 1e-12, (L, n_mu, got, want)


# ------------------------------------------------------- Eq. 17, binning


def test_p11_convolution_invariants():
    """P11: delta profile -> identity; constant -> constant (renormalised, also at
    the window edges); linear -> linear where the kernel fits in the window;
    the kernel's variance is that of a Gaussian of FWHM nu/R truncated at 5 sigma."""
    rng = np.random.default_rng(29)
    N, first, dnu = 4000, 3000.0, 0.5
    F = rng.uniform(0.5, 2.0, N)
    np.testing.assert_array_equal(oracle.convolve(F, first, dnu, 1e12), F)
    np.testing.assert_allclose(oracle.convolve(np.full(N, 3.25), first, dnu, 300.0), 3.25,
                               rtol=1e-14)
    nu = first + dnu * np.arange(N)
    R = 300.0
    out = oracle.convolve(2.0 + 1e-3 * nu, first, dnu, R)
    h_max = int(5 * nu[-1] / (R * 2 * np.sqrt(2 * np.log(2))) / dnu) + 1
    inner = slice(h_max, N - h_max)
    np.testing.assert_allclose(out[inner], (2.0 + 1e-3 * nu)[inner], rtol=1e-13)
    i = N // 2
    q = oracle.convolve((nu - nu[i]) ** 2, first, dnu, R, [i])[0]
    sig = nu[i] / (R * 2 * np.sqrt(2 * np.log(2)))
    z = 5.0
    trunc = 1 - 2 * z * np.exp(-z * z / 2) / np.sqrt(2 * np.pi) / special.erf(z / np.sqrt(2))
    assert abs(q / (sig * sig * trunc) - 1) < 2e-4
    # banded and full-window forms agree exactly
    idx = np.array([0, 5, 1999, N - 1])
    np.testing.assert_array_equal(oracle.convolve(F, first, dnu, R, idx, banded=True),
                                  oracle.convolve(F, first, dnu, R, idx, banded=False))


def test_p12_binning_exact_for_constant_and_linear():
    """P12: the trapezoid bin mean is exact for linear spectra; P13: linear in scale."""
    N, first, dnu = 500, 1000.0, 0.25
    nu = first + dnu * np.arange(N)
    edges = np.array([3, 40, 41, 77, 300, 499])
    b = oracle.bin_spectrum(np.full(N, 7.5), edges, first, dnu, 1.0)
    np.testing.assert_allclose(b, 7.5, rtol=1e-15)
    lin = 0.3 + 2e-3 * nu
    b = oracle.bin_spectrum(lin, edges, first, dnu, 1.0)
    want = 0.3 + 2e-3 * 0.5 * (nu[edges[:-1]] + nu[edges[1:]])
    np.testing.assert_allclose(b, want, rtol=1e-14)
    b2 = oracle.bin_spectrum(lin, edges, first, dnu, 2.0)
    np.testing.assert_array_equal(b2, 2.0 * b)


def test_edge_snapping_rule():
    idx = oracle.snap_edges([1000.1, 1000.25, 1001.9], 1000.0, 0.5, 10)
    np.testing.assert_array_equal(idx, [0, 1, 4])
    with pytest.raises(ValueError):
        oracle.snap_edges([1000.0, 1000.1], 1000.0, 0.5, 10)   # both snap to 0
    with pytest.raises(ValueError):
        oracle.snap_edges([1000.0, 1010.0], 1000.0, 0.5, 10)   # leaves the window


def test_p13_scale_and_subset_composition(c1):
    """The bin subset path equals the full chain; bins are linear in f (R/d)^2."""
    cols = wl.c1_columns()
    obs = wl.c1_obs(c1)
    full = oracle.forward(c1, cols[2], obs.window, obs.resolving_power, obs.edges_cm, 3)
    ids = [0, 17, 49]
    sub = oracle.forward_bins_subset(c1, cols[2], obs.window, obs.resolving_power, obs.edges_cm, 3,
                                     ids)
    np.testing.assert_allclose(sub, full["bins"][ids], rtol=1e-14)
    assert np.all(np.isfinite(full["bins"])) and np.all(full["bins"] > 0)
    col2 = wl.Column(cols[2].p_bar, cols[2].T_K, cols[2].x, cols[2].log_g, 3.0 * cols[2].scale)
    full2 = oracle.forward(c1, col2, obs.window, obs.resolving_power, obs.edges_cm, 3)
    np.testing.assert_allclose(full2["bins"], 3.0 * full["bins"], rtol=1e-15)


def test_hydrostatic_thickness_exact_for_t_linear_in_log_p():
    """Hydrostatic equilibrium of an ideal gas, dz = -k_B T / (mubar m_u g) dln p,
    integrated exactly for T linear in ln p: the layer thickness then equals
    k_B (T_l + T_l+1)/2 / (mubar m_u g) ln(p_l / p_l+1), so the column height is
    (k_B / mubar m_u g) int T dln p in closed form."""
    table = wl.c1_table()
    L = 41
    p = wl.levels(L, 2.0, -4.0)
    T0, T1 = 1450.0, 420.0
    lnp = np.log(p)
    T = T0 + (T1 - T0) * (lnp[0] - lnp) / (lnp[0] - lnp[-1])
    col = wl.Column(p, T, np.array([3e-3]), 5.1, 1.0)
    st = oracle.column_state(table, col)
    g = 10.0 ** 5.1
    height = np.cumsum(st["dz"])
    # int_{ln p_k}^{ln p_0} T dln p for T linear in ln p
    s = lnp[0] - lnp[1:]
    integral = T0 * s + (T1 - T0) * s * s / (2 * (lnp[0] - lnp[-1]))
    want = KB * integral / (st["mubar"] * AMU * g)
    np.testing.assert_allclose(height, want, rtol=AMU_RTOL)


# ------------------------------------------------------------ Eq. 19, 22-23


def test_likelihood_matches_the_gaussian_density():
    """Eq. 19 is the log of a product of normal densities: it equals the sum of
    scipy's norm.logpdf; with error inflation (Eq. 22-23) the scale becomes
    sqrt(sigma^2 + 10^eps)."""
    from scipy import stats
    rng = np.random.default_rng(31)
    m = rng.uniform(1.0, 5.0, 57)
    sg = rng.uniform(0.05, 0.5, 57)
    D = m + sg * rng.normal(size=57)
    want = np.sum(stats.norm.logpdf(D, loc=m, scale=sg))
    assert abs(oracle.log_likelihood(m, D, sg) - want) < 1e-12 * abs(want)
    eps = -1.7
    want = np.sum(stats.norm.logpdf(D, loc=m, scale=np.sqrt(sg ** 2 + 10.0 ** eps)))
    assert abs(oracle.log_likelihood(m, D, sg, eps) - want) < 1e-12 * abs(want)
    # a perfect model leaves only the normalisation
    assert abs(oracle.log_likelihood(m, m, sg) + 0.5 * np.sum(np.log(2 * np.pi * sg ** 2))) < 1e-12
