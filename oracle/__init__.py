"""FP64 CPU oracle of the Helios-r2 emission forward model (arXiv:1910.01070).

TEST INFRASTRUCTURE ONLY: the tests, the package smoke check and the
benchmark's CPU-baseline leg call it; the product path never does.  It shares
no code with the HIP library and imports nothing from it.

Thin ctypes wrapper around ``hr2_oracle.c`` plus the composition of its
stages (opacity -> RT -> convolution -> binning) for a column.  Inputs are
duck-typed: a table needs ``T_K, log10_p_bar, nu0_cm, dnu_cm, n_nu,
log10_sigma, molar_mass, log10_k_cia, he_h2_ratio``; a column ``p_bar, T_K,
x, log_g, scale`` and optionally ``cloud`` = (tau_c, p_top_bar, bottom_frac)
or None (App. B); a window ``begin, count, stride``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# HR2_ORACLE_LIB: another build of hr2_oracle.c (the sanitizer test's)
LIB_PATH = os.environ.get("HR2_ORACLE_LIB", os.path.join(HERE, "liboracle.so"))

_D = ctypes.c_double
_DP = ctypes.POINTER(ctypes.c_double)
_I64 = ctypes.c_int64
_I64P = ctypes.POINTER(ctypes.c_int64)
_I = ctypes.c_int


def build(force: bool = True) -> str:
    if force or not os.path.exists(LIB_PATH):
        tmp = LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", tmp,
                               os.path.join(HERE, "hr2_oracle.c"), "-lm"])
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


_handle = None


def lib():
    global _handle
    if _handle is None:
        src = os.path.join(HERE, "hr2_oracle.c")
        if "HR2_ORACLE_LIB" not in os.environ and (
                not os.path.exists(LIB_PATH) or os.path.getmtime(src) > os.path.getmtime(LIB_PATH)):
            build(force=True)
        L = ctypes.CDLL(LIB_PATH)
        L.or_set_threads.argtypes = [_I]
        L.or_set_threads.restype = None
        L.or_max_threads.argtypes = []
        L.or_max_threads.restype = _I
        L.or_gauss_legendre01.argtypes = [_I, _DP, _DP]
        L.or_gauss_legendre01.restype = _I
        L.or_planck.argtypes = [_D, _D]
        L.or_planck.restype = _D
        L.or_planck_n.argtypes = [_I64, _DP, _DP, _DP]
        L.or_planck_n.restype = None
        L.or_column_state.argtypes = [_I, _DP, _DP, _I, _DP, _DP, _D, _D, _DP, _DP, _DP, _DP, _DP]
        L.or_column_state.restype = None
        L.or_opacity.argtypes = [_I, _I, _I, _DP, _DP, _I64, _DP, _I, _DP, _DP, _D, _I, _DP, _DP,
                                 _DP, _D, _I64, _I64P, _DP]
        L.or_opacity.restype = None
        L.or_sc_intensity.argtypes = [_I, _DP, _DP, _D]
        L.or_sc_intensity.restype = _D
        L.or_sc_flux.argtypes = [_I, _DP, _DP, _I]
        L.or_sc_flux.restype = _D
        L.or_rt_emission.argtypes = [_I, _I64, _DP, _DP, _DP, _DP, _I, _DP]
        L.or_rt_emission.restype = None
        L.or_rt_emission_x.argtypes = [_I, _I64, _DP, _DP, _DP, _DP, _I, _DP, _DP]
        L.or_rt_emission_x.restype = None
        L.or_cloud_dtau.argtypes = [_I, _DP, _D, _D, _D, _DP]
        L.or_cloud_dtau.restype = None
        L.or_rt_emission_o.argtypes = [_I, _I64, _DP, _DP, _DP, _DP, _I, _DP, _I, _DP]
        L.or_rt_emission_o.restype = None
        L.or_sc_para_coeffs.argtypes = [_D, _D, _DP, _DP, _DP]
        L.or_sc_para_coeffs.restype = None
        L.or_sc_intensity_para.argtypes = [_I, _DP, _DP, _D]
        L.or_sc_intensity_para.restype = _D
        L.or_sc_flux_o.argtypes = [_I, _DP, _DP, _I, _I]
        L.or_sc_flux_o.restype = _D
        for name in ("or_convolve", "or_convolve_banded"):
            fn = getattr(L, name)
            fn.argtypes = [_I64, _D, _D, _DP, _D, _I64, _I64P, _DP]
            fn.restype = None
        L.or_snap_edges.argtypes = [_I, _DP, _D, _D, _I64, _I64P]
        L.or_snap_edges.restype = _I
        L.or_bin.argtypes = [_D, _D, _DP, _I, _I64P, _D, _DP]
        L.or_bin.restype = None
        L.or_lnl.argtypes = [_I, _DP, _DP, _DP, _I, _D]
        L.or_lnl.restype = _D
        _handle = L
    return _handle


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _i64(a):
    return np.ascontiguousarray(a, dtype=np.int64)


def _p(a):
    if a.dtype == np.int64:
        return a.ctypes.data_as(_I64P)
    return a.ctypes.data_as(_DP)


# ------------------------------------------------------------------ pieces


def gauss_legendre01(n):
    mu = np.empty(n)
    w = np.empty(n)
    if lib().or_gauss_legendre01(int(n), _p(mu), _p(w)) != 0:
        raise ValueError("n must be >= 1")
    return mu, w


def planck(nu_cm, T_K):
    shape = np.broadcast_shapes(np.shape(nu_cm), np.shape(T_K))
    nu = _f64(np.broadcast_to(np.asarray(nu_cm, dtype=np.float64), shape).ravel())
    T = _f64(np.broadcast_to(np.asarray(T_K, dtype=np.float64), shape).ravel())
    out = np.empty(nu.size)
    lib().or_planck_n(nu.size, _p(nu), _p(T), _p(out))
    return out.reshape(shape)


def column_state(table, col):
    p, T, x = _f64(col.p_bar), _f64(col.T_K), _f64(col.x)
    L = len(p)
    n_tot = np.empty(L)
    dz = np.empty(max(L - 1, 1))
    xh2, xhe, mub = _D(), _D(), _D()
    lib().or_column_state(L, _p(p), _p(T), len(x), _p(x), _p(_f64(table.molar_mass)),
                          float(table.he_h2_ratio), float(col.log_g), _p(n_tot),
                          ctypes.byref(xh2), ctypes.byref(xhe), ctypes.byref(mub), _p(dz))
    return dict(n_tot=n_tot, x_h2=xh2.value, x_he=xhe.value, mubar=mub.value, dz=dz[:L - 1])


def window_indices(window):
    return window.begin + window.stride * np.arange(window.count, dtype=np.int64)


def opacity(table, col, nu_idx):
    """chi[L][len(nu_idx)] at table wavenumber indices nu_idx."""
    nu_idx = _i64(nu_idx)
    p, T, x = _f64(col.p_bar), _f64(col.T_K), _f64(col.x)
    L = len(p)
    sig = table.log10_sigma
    assert sig.dtype == np.float64 and sig.flags.c_contiguous
    S, nT, nP, n_nu = sig.shape
    cia = table.log10_k_cia
    n_cia = 0 if cia is None else cia.shape[0]
    cia_arr = _f64(cia) if cia is not None else np.zeros(1)
    chi = np.empty((L, len(nu_idx)))
    lib().or_opacity(S, nT, nP, _p(_f64(table.T_K)), _p(_f64(table.log10_p_bar)), n_nu, _p(sig),
                     n_cia, _p(cia_arr), _p(_f64(table.molar_mass)), float(table.he_h2_ratio), L,
                     _p(p), _p(T), _p(x), float(col.log_g), len(nu_idx), _p(nu_idx), _p(chi))
    return chi


def sc_intensity(dtau, S, mu):
    dtau, S = _f64(dtau), _f64(S)
    return lib().or_sc_intensity(len(S), _p(dtau), _p(S), float(mu))


def sc_flux(dtau, S, n_mu, order=1):
    dtau, S = _f64(dtau), _f64(S)
    return lib().or_sc_flux_o(len(S), _p(dtau), _p(S), int(n_mu), int(order))


def sc_para_coeffs(du, dd):
    """(alpha, beta, gamma) of the parabolic step for path lengths du, dd."""
    a, b, g = _D(), _D(), _D()
    lib().or_sc_para_coeffs(float(du), float(dd), ctypes.byref(a), ctypes.byref(b),
                            ctypes.byref(g))
    return a.value, b.value, g.value


def sc_intensity_para(dtau, S, mu):
    dtau, S = _f64(dtau), _f64(S)
    return lib().or_sc_intensity_para(len(S), _p(dtau), _p(S), float(mu))


def cloud_dtau(p_bar, cloud):
    """Per-layer optical depth of a gray cloud (tau_c, p_top_bar, bottom_frac), App. B."""
    p = _f64(p_bar)
    out = np.empty(max(len(p) - 1, 1))
    tau_c, p_top, frac = cloud
    lib().or_cloud_dtau(len(p), _p(p), float(tau_c), float(p_top), float(frac), _p(out))
    return out[:len(p) - 1]


def rt_emission(chi, dz, T_K, nu, n_mu, dtau_extra=None, order=1):
    """F+ (Eq. 2-8); order 1: linear source, order 2: parabolic source."""
    chi = _f64(chi)
    L, n = chi.shape
    out = np.empty(n)
    if dtau_extra is None and order == 1:
        lib().or_rt_emission(L, n, _p(chi), _p(_f64(dz)), _p(_f64(T_K)), _p(_f64(nu)), int(n_mu),
                             _p(out))
    else:
        ex = None if dtau_extra is None else _f64(dtau_extra)
        lib().or_rt_emission_o(L, n, _p(chi), _p(_f64(dz)), _p(_f64(T_K)), _p(_f64(nu)),
                               int(n_mu), None if ex is None else _p(ex), int(order), _p(out))
    return out


def convolve(F, nu_first, dnu_eff, R, out_idx=None, banded=True):
    F = _f64(F)
    N = len(F)
    out_idx = np.arange(N, dtype=np.int64) if out_idx is None else _i64(out_idx)
    out = np.empty(len(out_idx))
    fn = lib().or_convolve_banded if banded else lib().or_convolve
    fn(N, float(nu_first), float(dnu_eff), _p(F), float(R), len(out_idx), _p(out_idx), _p(out))
    return out


def snap_edges(edges_cm, nu_first, dnu_eff, N):
    e = _f64(edges_cm)
    idx = np.empty(len(e), dtype=np.int64)
    if lib().or_snap_edges(len(e), _p(e), float(nu_first), float(dnu_eff), int(N), _p(idx)) != 0:
        raise ValueError("bin edges leave the window or are not strictly increasing")
    return idx


def bin_spectrum(Fd, edge_idx, nu_first, dnu_eff, scale):
    Fd, edge_idx = _f64(Fd), _i64(edge_idx)
    nb = len(edge_idx) - 1
    out = np.empty(nb)
    lib().or_bin(float(nu_first), float(dnu_eff), _p(Fd), nb, _p(edge_idx), float(scale), _p(out))
    return out


def log_likelihood(model, D, sigma, log10_eps=None):
    """Eq. 19, or Eq. 22-23 with s^2 = sigma^2 + 10^eps when log10_eps is given."""
    m, D, sg = _f64(model), _f64(D), _f64(sigma)
    return lib().or_lnl(len(m), _p(m), _p(D), _p(sg), 0 if log10_eps is None else 1,
                        0.0 if log10_eps is None else float(log10_eps))


def set_threads(n):
    """Threads of the oracle's OpenMP loops (for timing; results do not change)."""
    lib().or_set_threads(int(n))


def max_threads():
    return int(lib().or_max_threads())


# ------------------------------------------------------------- composition


def window_grid(table, window):
    nu_first = table.nu0_cm + window.begin * table.dnu_cm
    dnu_eff = window.stride * table.dnu_cm
    return nu_first, dnu_eff


def fplus(table, col, window, n_mu, sub=None, order=1):
    """F+ at window points ``sub`` (all when None): opacity then RT."""
    idx_w = np.arange(window.count, dtype=np.int64) if sub is None else _i64(sub)
    tab_idx = window.begin + window.stride * idx_w
    chi = opacity(table, col, tab_idx)
    st = column_state(table, col)
    nu = table.nu0_cm + tab_idx * table.dnu_cm
    cloud = getattr(col, "cloud", None)
    extra = None if cloud is None else cloud_dtau(col.p_bar, cloud)
    return rt_emission(chi, st["dz"], col.T_K, nu, n_mu, extra, order)


def forward(table, col, window, R, edges_cm, n_mu, order=1):
    """Whole chain on the full window: dict with fplus, fd and bins."""
    nu_first, dnu_eff = window_grid(table, window)
    fp = fplus(table, col, window, n_mu, order=order)
    edge_idx = snap_edges(edges_cm, nu_first, dnu_eff, window.count)
    a, b = int(edge_idx[0]), int(edge_idx[-1])
    fd = np.full(window.count, np.nan)
    fd[a:b + 1] = convolve(fp, nu_first, dnu_eff, R, np.arange(a, b + 1))
    bins = bin_spectrum(fd, edge_idx, nu_first, dnu_eff, col.scale)
    return dict(fplus=fp, fd=fd, bins=bins, edge_idx=edge_idx)


def half_width(nu_first, dnu_eff, R, i):
    """Largest k with k dnu_eff <= 5 sigma_i (the 5 sigma cut of the convolution)."""
    sig = (nu_first + i * dnu_eff) / (R * 2.0 * np.sqrt(2.0 * np.log(2.0)))
    h = int(5.0 * sig / dnu_eff) + 2
    while h > 0 and h * dnu_eff > 5.0 * sig:
        h -= 1
    return h


def forward_bins_subset(table, col, window, R, edges_cm, n_mu, bin_ids, order=1):
    """Selected bins only: F+ on each bin's support, convolution on the bin's points."""
    nu_first, dnu_eff = window_grid(table, window)
    edge_idx = snap_edges(edges_cm, nu_first, dnu_eff, window.count)
    out = np.empty(len(bin_ids))
    for q, j in enumerate(bin_ids):
        a, b = int(edge_idx[j]), int(edge_idx[j + 1])
        lo = max(0, a - half_width(nu_first, dnu_eff, R, a) - 1)
        hi = min(window.count - 1, b + half_width(nu_first, dnu_eff, R, b) + 1)
        sub = np.arange(lo, hi + 1, dtype=np.int64)
        fp_sub = fplus(table, col, window, n_mu, sub, order)
        fp_full = np.zeros(window.count)
        fp_full[lo:hi + 1] = fp_sub
        fd = np.zeros(window.count)
        fd[a:b + 1] = convolve(fp_full, nu_first, dnu_eff, R, np.arange(a, b + 1))
        out[q] = bin_spectrum(fd, np.array([a, b]), nu_first, dnu_eff, col.scale)[0]
    return out
