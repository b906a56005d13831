"""Oracle of the parameter-to-column step (FP64, plain numpy; TEST
INFRASTRUCTURE ONLY, like the rest of this package).

Finite-element temperature profile (Sect. 2.5.1, Eq. 12-16): K_e elements of
order q split the log-pressure range of the model atmosphere into equal
parts; on each element the temperature is the Lagrange interpolant (Eq. 13)
through q + 1 nodes placed at the Gauss-Lobatto points of the reference
element [0, 1]; neighbouring elements share their boundary node (continuous
form), so there are N_T = K_e q + 1 node temperatures (Eq. 16).  Only the
bottom node's temperature is a parameter; every further node is b times the
node below it.

Free chemistry (Sect. 5.2): height-independent mixing ratios; a species not
retrieved directly may be a fixed multiple of a retrieved one (sodium from
potassium); H2 and He fill the rest, which the forward model already does.

Radius-distance factor (Eq. 9): scale = f (R_* / d)^2.

Gray cloud (App. B), optional: optical depth, top pressure and the bottom as
a multiple of the top, passed on with the column.

Readings taken where the paper is silent:
* elements and levels span the same log-pressure range, element 1 at the
  bottom, local coordinate 0 at each element's bottom boundary;
* node n (counted from the bottom, from 0) has T_n = b_n T_{n-1};
* a level on an element boundary takes the element above it (both give the
  same temperature, the profile being continuous);
* the distance parameter is in parsec.
"""
from __future__ import annotations

import numpy as np

PARSEC_CM = 3.0856775814913673e18


def gauss_lobatto01(n_points: int) -> np.ndarray:
    """The n_points Gauss-Lobatto nodes on [0, 1]: both ends plus the roots of
    P'_{n-1}, the derivative of the Legendre polynomial of degree n - 1."""
    if n_points < 2:
        raise ValueError("need at least the two end points")
    q = n_points - 1
    inner = np.polynomial.legendre.Legendre.basis(q).deriv().roots() if q >= 2 else np.array([])
    x = np.concatenate([[-1.0], np.sort(np.real(inner)), [1.0]])
    return 0.5 * (x + 1.0)


def lagrange_basis(nodes: np.ndarray, xi: float) -> np.ndarray:
    """Eq. 13: l_i(xi) = prod_{j != i} (xi - x_j) / (x_i - x_j)."""
    out = np.ones(len(nodes))
    for i in range(len(nodes)):
        for j in range(len(nodes)):
            if j != i:
                out[i] *= (xi - nodes[j]) / (nodes[i] - nodes[j])
    return out


def node_temperatures(T1: float, b) -> np.ndarray:
    """T_0 = T1 (the bottom node), T_n = b_n T_{n-1}."""
    T = [float(T1)]
    for bn in b:
        T.append(float(bn) * T[-1])
    return np.array(T)


def fe_temperature(log10_p, log10_p_bottom, log10_p_top, n_elements, order, T_nodes):
    """Eq. 12-15 at the pressures log10_p (bar): the global piecewise
    polynomial through the node temperatures T_nodes[K_e q + 1]."""
    T_nodes = np.asarray(T_nodes, dtype=np.float64)
    if len(T_nodes) != n_elements * order + 1:
        raise ValueError("Eq. 16: need K_e q + 1 node temperatures")
    nodes = gauss_lobatto01(order + 1)
    lp = np.atleast_1d(np.asarray(log10_p, dtype=np.float64))
    out = np.empty(len(lp))
    for m, x in enumerate(lp):
        u = (log10_p_bottom - x) / (log10_p_bottom - log10_p_top) * n_elements
        k = min(max(int(np.floor(u)), 0), n_elements - 1)
        xi = u - k
        out[m] = float(np.dot(T_nodes[k * order:(k + 1) * order + 1], lagrange_basis(nodes, xi)))
    return out


def level_pressures(n_levels, log10_p_bottom, log10_p_top):
    """Levels equidistant in log p, level 0 at the bottom (bar)."""
    return 10.0 ** np.linspace(log10_p_bottom, log10_p_top, n_levels)


def _with_cloud(layout) -> bool:
    return bool(getattr(layout, "with_cloud", False))


def n_theta(layout) -> int:
    """Parameters per set: log g, f, d, T1, the N_T - 1 b's, the free mixing
    ratios, the three gray-cloud parameters (App. B) when the layout has a
    cloud, and log10 eps when it carries one."""
    return (3 + layout.n_elements * layout.order + 1 + layout.n_free + 3 * _with_cloud(layout)
            + int(layout.with_eps))


def unpack(layout, theta):
    """One parameter vector -> (p_bar, T_K, x, log_g, scale, cloud or None,
    log10_eps or None); cloud = (tau_c, p_top_bar, bottom_frac)."""
    th = np.asarray(theta, dtype=np.float64)
    if len(th) != n_theta(layout):
        raise ValueError("wrong parameter count")
    log_g, f, d_pc, T1 = th[0], th[1], th[2], th[3]
    NT = layout.n_elements * layout.order + 1
    b = th[4:3 + NT]
    xf = th[3 + NT:3 + NT + layout.n_free]
    k = 3 + NT + layout.n_free
    cloud = tuple(float(v) for v in th[k:k + 3]) if _with_cloud(layout) else None
    k += 3 * _with_cloud(layout)
    eps = float(th[k]) if layout.with_eps else None
    p = level_pressures(layout.n_levels, layout.log10_p_bottom, layout.log10_p_top)
    T = fe_temperature(np.log10(p), layout.log10_p_bottom, layout.log10_p_top,
                       layout.n_elements, layout.order, node_temperatures(T1, b))
    src = np.asarray(layout.species_src)
    fac = np.asarray(layout.species_factor, dtype=np.float64)
    x = np.array([fac[s] * xf[src[s]] if src[s] >= 0 else 0.0 for s in range(len(src))])
    scale = f * (layout.radius_cm / (d_pc * PARSEC_CM)) ** 2
    return p, T, x, float(log_g), float(scale), cloud, eps
