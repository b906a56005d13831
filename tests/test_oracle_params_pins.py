"""Pins of the parameter-to-column oracle (finite-element temperature
profile, Sect. 2.5.1, Eq. 12-16; free chemistry, Sect. 5.2; Eq. 9).

Expected values come from textbook closed forms of the Gauss-Lobatto nodes,
from exactness properties of Lagrange interpolation (nodal values, partition
of unity, reproduction of polynomials up to the element order), from the
parameter counts the paper states, and from the radius-distance factor
worked out by hand."""
import numpy as np
import pytest

from oracle import params as op
import workloads as wl


@pytest.mark.parametrize("n,want", [
    (2, [0.0, 1.0]),
    (3, [0.0, 0.5, 1.0]),
    (4, [0.0, 0.5 * (1 - 1 / np.sqrt(5)), 0.5 * (1 + 1 / np.sqrt(5)), 1.0]),
    (5, [0.0, 0.5 * (1 - np.sqrt(3 / 7)), 0.5, 0.5 * (1 + np.sqrt(3 / 7)), 1.0]),
    (6, [0.0, 0.5 * (1 - np.sqrt(1 / 3 + 2 * np.sqrt(7) / 21)),
         0.5 * (1 - np.sqrt(1 / 3 - 2 * np.sqrt(7) / 21)),
         0.5 * (1 + np.sqrt(1 / 3 - 2 * np.sqrt(7) / 21)),
         0.5 * (1 + np.sqrt(1 / 3 + 2 * np.sqrt(7) / 21)), 1.0]),
])
def test_gauss_lobatto_nodes_closed_forms(n, want):
    """Gauss-Lobatto points on [-1, 1] (Abramowitz & Stegun 25.4.32 table),
    mapped to the reference element [0, 1]."""
    assert np.allclose(op.gauss_lobatto01(n), want, rtol=0, atol=1e-14)


def test_gauss_lobatto_quadrature_exactness():
    """With Lobatto weights w_i = 2 / (n (n-1) P_{n-1}(x_i)^2) the nodes
    integrate polynomials up to degree 2n - 3 exactly: a wrong node fails."""
    for n in range(3, 9):
        x = 2.0 * op.gauss_lobatto01(n) - 1.0
        P = np.polynomial.legendre.Legendre.basis(n - 1)(x)
        w = 2.0 / (n * (n - 1) * P * P)
        for deg in range(0, 2 * n - 2):
            exact = 0.0 if deg % 2 else 2.0 / (deg + 1)
            assert abs(np.sum(w * x ** deg) - exact) < 1e-13


@pytest.mark.parametrize("q", [1, 2, 3, 5])
def test_lagrange_nodal_and_partition_of_unity(q):
    nodes = op.gauss_lobatto01(q + 1)
    for j, xj in enumerate(nodes):
        l = op.lagrange_basis(nodes, xj)
        assert np.allclose(l, np.eye(q + 1)[j], atol=1e-14)
    for xi in np.linspace(0, 1, 17):
        assert abs(op.lagrange_basis(nodes, xi).sum() - 1.0) < 1e-13


@pytest.mark.parametrize("K,q", [(1, 1), (6, 1), (3, 2), (4, 3), (2, 4)])
def test_fe_reproduces_polynomials_up_to_order(K, q):
    """Node temperatures sampled from a polynomial of degree <= q in log p
    give back that polynomial everywhere (Eq. 12-15), on every element."""
    lpb, lpt = 2.5, -5.0
    rng = np.random.default_rng(K * 10 + q)
    coef = rng.uniform(-1, 1, q + 1)
    poly = lambda lp: 1500.0 + 100.0 * np.polynomial.polynomial.polyval((lp - lpt) / (lpb - lpt),
                                                                          coef)
    nodes = op.gauss_lobatto01(q + 1)
    node_lp = [lpb - (k + nodes[i]) / K * (lpb - lpt) for k in range(K) for i in range(q)]
    node_lp.append(lpt)
    Tn = poly(np.array(node_lp))
    lp = np.linspace(lpb, lpt, 203)
    got = op.fe_temperature(lp, lpb, lpt, K, q, Tn)
    assert np.max(np.abs(got - poly(lp))) < 1e-9
    # and at the nodes themselves the interpolant returns the node values
    assert np.allclose(op.fe_temperature(np.array(node_lp), lpb, lpt, K, q, Tn), Tn,
                       rtol=1e-13)


def test_fe_profile_is_continuous_and_monotone():
    """Continuous across element boundaries (the shared node); with q = 1 and
    b <= 1 the profile never increases with height."""
    lpb, lpt, K = 3.0, -6.0, 6
    Tn = op.node_temperatures(2500.0, [0.9, 0.8, 0.95, 0.7, 0.85, 0.9])
    for k in range(1, K):
        lb = lpb - k / K * (lpb - lpt)
        lo, hi = op.fe_temperature(np.array([lb + 1e-12, lb - 1e-12]), lpb, lpt, K, 1, Tn)
        assert abs(lo - hi) < 1e-6
    T = op.fe_temperature(np.linspace(lpb, lpt, 301), lpb, lpt, K, 1, Tn)
    assert np.all(np.diff(T) <= 1e-12)
    # second-order elements with all b = 1: isothermal
    Ti = op.node_temperatures(1234.5, np.ones(6))
    assert np.allclose(op.fe_temperature(np.linspace(lpb, lpt, 50), lpb, lpt, 3, 2, Ti), 1234.5,
                       rtol=1e-14)


def test_first_order_midpoint_is_the_node_mean():
    Tn = op.node_temperatures(2000.0, [0.5])
    assert abs(op.fe_temperature(np.array([0.0]), 1.0, -1.0, 1, 1, Tn)[0] - 1500.0) < 1e-12


def test_parameter_counts_match_the_paper():
    """Eq. 16: N_T = K_e q + 1; six first-order or three second-order elements
    both give seven temperature parameters, and the free-chemistry retrieval
    has 18 parameters in all (Sect. 5.2): log g, d, f, T1, six b, seven x, eps."""
    for K, q in ((6, 1), (3, 2)):
        lay = wl.c2_param_layout(K, q, with_eps=True)
        assert K * q + 1 == 7
        assert op.n_theta(lay) == 18


def test_unpack_scale_mixing_ratios_and_levels():
    lay = wl.c2_param_layout(3, 2, with_eps=True)
    th = wl.draw_theta(lay, 1, seed=4)[0]
    th[1], th[2] = 2.0, 10.0                      # f = 2, d = 10 pc
    p, T, x, lg, scale, cloud, eps = op.unpack(lay, th)
    # f (R_J / 10 pc)^2 by hand: 7.1492e9 / 3.0856775814913673e19 = 2.31690...e-10
    assert abs(scale - 2.0 * (7.1492e9 / 3.0856775814913673e19) ** 2) < 1e-28
    assert abs(scale / 1.0736e-19 - 1.0) < 1e-3
    assert np.allclose(x[:7], th[10:17], rtol=0) and abs(x[7] - wl.SOLAR_NA_K * th[16]) < 1e-20
    assert len(p) == 101 and abs(p[0] - 1e3) < 1e-9 and abs(p[-1] - 1e-6) < 1e-18
    assert np.allclose(np.diff(np.log10(p)), -0.09, atol=1e-12)
    assert T[0] == th[3] and eps == th[-1] and lg == th[0]
    # the top level is the last node: T1 times every b
    assert abs(T[-1] - th[3] * np.prod(th[4:10])) < 1e-9
