"""Seeded synthetic inputs for the Helios-r2 forward model.

Input generation only: this module draws line lists, atmospheric columns,
observation layouts and serving traces from seeded numpy generators (PCG64)
and evaluates synthetic cross-section tables with ``gen_xsec.c``.  It holds
none of the forward model's arithmetic; both the oracle and the HIP path
consume what it returns.

The shapes follow the paper's workloads: 70-level log-p grids (Sect. 2),
1 cm^-1 and finer wavenumber steps (Sect. 2.1, 2.8), the absorbers of
Sect. 2.3 with H2-H2 / H2-He CIA, the priors of Table 1 (log g, f, b_i, T_1,
log-uniform abundances), R_* = 1 R_J and d = 10 pc (Sect. 2.2, 4), and about
150-400 observational bins (Sect. 4.1, 5.1).  The paper's own data (line
lists, CIA tables, observed spectra) are replaced by these stand-ins.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field
from typing import List, Optional, Tuple

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgen_xsec.so")

R_JUP_CM = 7.1492e9
PARSEC_CM = 3.0856775814913673e18
HE_H2_RATIO = 0.17

SPECIES_MASS = {
    "H2O": 18.015, "CH4": 16.043, "CO": 28.010, "CO2": 44.009,
    "NH3": 17.031, "H2S": 34.08, "K": 39.098, "Na": 22.990, "X": 30.0,
}


def build_generator(force: bool = True) -> str:
    """Compile gen_xsec.c into a shared library next to it."""
    if force or not os.path.exists(LIB_PATH):
        src = os.path.join(HERE, "gen_xsec.c")
        tmp = LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O3", "-fopenmp", "-fPIC", "-shared", "-o", tmp, src, "-lm"])
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


_lib_handle = None


def _lib():
    global _lib_handle
    if _lib_handle is None:
        if not os.path.exists(LIB_PATH):
            build_generator(force=True)
        lib = ctypes.CDLL(LIB_PATH)
        dp = ctypes.POINTER(ctypes.c_double)
        lib.gen_xsec_table.argtypes = [
            ctypes.c_int, dp, dp, dp, dp, ctypes.c_double,
            ctypes.c_int, dp, ctypes.c_int, dp,
            ctypes.c_double, ctypes.c_double, ctypes.c_int64, ctypes.c_double,
            ctypes.c_double, dp]
        lib.gen_xsec_table.restype = None
        _lib_handle = lib
    return _lib_handle


def _dp(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


# --------------------------------------------------------------------------- data


@dataclass
class Table:
    T_K: np.ndarray                 # [n_T]
    log10_p_bar: np.ndarray         # [n_p]
    nu0_cm: float
    dnu_cm: float
    n_nu: int
    log10_sigma: np.ndarray         # [S][n_T][n_p][n_nu] float64
    molar_mass: np.ndarray          # [S]
    log10_k_cia: Optional[np.ndarray] = None   # [2][n_T][n_nu] or None
    he_h2_ratio: float = HE_H2_RATIO
    species: List[str] = field(default_factory=list)

    @property
    def n_species(self) -> int:
        return int(self.log10_sigma.shape[0])

    @property
    def n_cia(self) -> int:
        return 0 if self.log10_k_cia is None else int(self.log10_k_cia.shape[0])

    def nu(self, begin=0, count=None, stride=1) -> np.ndarray:
        if count is None:
            count = (self.n_nu - begin + stride - 1) // stride
        k = begin + stride * np.arange(count, dtype=np.int64)
        return self.nu0_cm + k * self.dnu_cm


@dataclass
class Column:
    p_bar: np.ndarray    # [L], decreasing
    T_K: np.ndarray      # [L]
    x: np.ndarray        # [S]
    log_g: float
    scale: float
    cloud: Optional[Tuple[float, float, float]] = None   # (tau_c, p_top_bar, bottom_frac)

    @property
    def n_levels(self) -> int:
        return int(self.p_bar.shape[0])


@dataclass
class Window:
    begin: int
    count: int
    stride: int = 1


@dataclass
class ObsSpec:
    window: Window
    resolving_power: float
    edges_cm: np.ndarray  # [n_bins + 1]

    @property
    def n_bins(self) -> int:
        return int(self.edges_cm.shape[0] - 1)


# ---------------------------------------------------------------- line lists


def line_list_uniform(rng, n_lines, nu_lo, nu_hi, s_lo, s_hi):
    nu = rng.uniform(nu_lo, nu_hi, n_lines)
    s = 10.0 ** rng.uniform(np.log10(s_lo), np.log10(s_hi), n_lines)
    e = rng.uniform(0.0, 3000.0, n_lines)
    g = rng.uniform(0.03, 0.1, n_lines)
    return nu, s, e, g


def line_list_bands(rng, n_lines, nu_lo, nu_hi, s_lo, s_hi, n_bands=3):
    centers = rng.uniform(nu_lo + 0.05 * (nu_hi - nu_lo), nu_hi - 0.05 * (nu_hi - nu_lo), n_bands)
    widths = rng.uniform(300.0, 1500.0, n_bands)
    which = rng.integers(0, n_bands, n_lines)
    nu = rng.normal(centers[which], widths[which])
    nu = np.clip(nu, nu_lo, nu_hi)
    s = 10.0 ** rng.uniform(np.log10(s_lo), np.log10(s_hi), n_lines)
    e = rng.uniform(0.0, 3000.0, n_lines)
    g = rng.uniform(0.03, 0.1, n_lines)
    return nu, s, e, g


def xsec_table(lines, mass, T_K, log10_p, nu0, dnu, n_nu, wing_cut=25.0, floor=1e-30):
    nu, s, e, g = (np.ascontiguousarray(a, dtype=np.float64) for a in lines)
    T_K = np.ascontiguousarray(T_K, dtype=np.float64)
    log10_p = np.ascontiguousarray(log10_p, dtype=np.float64)
    out = np.empty((len(T_K), len(log10_p), int(n_nu)), dtype=np.float64)
    _lib().gen_xsec_table(len(nu), _dp(nu), _dp(s), _dp(e), _dp(g), float(mass),
                          len(T_K), _dp(T_K), len(log10_p), _dp(log10_p),
                          float(nu0), float(dnu), int(n_nu), float(wing_cut), float(floor),
                          _dp(out))
    return out


def cia_table(rng, T_K, nu, floor=1e-60):
    """Smooth H2-H2 and H2-He continua: A (T/300)^0.5 sum_b exp(-(nu-nu_b)^2 / 2 w_b^2)."""
    amps = (1e-46, 3e-47)
    centers = np.array([0.0, 4162.0, 8089.0])
    out = np.empty((2, len(T_K), len(nu)), dtype=np.float64)
    for pair in range(2):
        widths = rng.uniform(300.0, 600.0, 3)
        shape = np.zeros_like(nu)
        for c, w in zip(centers, widths):
            shape += np.exp(-(nu - c) ** 2 / (2.0 * w * w))
        for it, T in enumerate(T_K):
            out[pair, it] = np.log10(floor + amps[pair] * np.sqrt(T / 300.0) * shape)
    return out


def make_table(seed, species, T_K, log10_p, nu0, dnu, n_nu, n_lines=200, bands=False,
               s_range=(1e-23, 1e-19), with_cia=False, wing_cut=25.0):
    """Generic seeded table; used by the configurations and by the tests."""
    rng = np.random.default_rng(seed)
    T_K = np.asarray(T_K, dtype=np.float64)
    log10_p = np.asarray(log10_p, dtype=np.float64)
    nu_hi = nu0 + (n_nu - 1) * dnu
    sig = np.empty((len(species), len(T_K), len(log10_p), int(n_nu)), dtype=np.float64)
    for i, sp in enumerate(species):
        if bands:
            lines = line_list_bands(rng, n_lines, nu0, nu_hi, *s_range)
        else:
            lines = line_list_uniform(rng, n_lines, nu0, nu_hi, *s_range)
        sig[i] = xsec_table(lines, SPECIES_MASS.get(sp, 30.0), T_K, log10_p, nu0, dnu, n_nu,
                            wing_cut=wing_cut)
    cia = None
    if with_cia:
        nu = nu0 + dnu * np.arange(n_nu, dtype=np.float64)
        cia = cia_table(rng, T_K, nu)
    return Table(T_K=T_K, log10_p_bar=log10_p, nu0_cm=float(nu0), dnu_cm=float(dnu),
                 n_nu=int(n_nu), log10_sigma=sig,
                 molar_mass=np.array([SPECIES_MASS.get(sp, 30.0) for sp in species]),
                 log10_k_cia=cia, species=list(species))


# ------------------------------------------------------------------ columns


def scale_factor(f, radius_cm=R_JUP_CM, distance_cm=10.0 * PARSEC_CM):
    return float(f) * (radius_cm / distance_cm) ** 2


def levels(n_levels, log10_p_bottom, log10_p_top):
    return 10.0 ** np.linspace(log10_p_bottom, log10_p_top, n_levels)


def linear_logp_profile(p_bar, T_bottom, T_top):
    lp = np.log10(p_bar)
    return T_bottom + (T_top - T_bottom) * (lp[0] - lp) / (lp[0] - lp[-1])


def piecewise_knot_profile(p_bar, T1, b):
    """First-order elements, knots equidistant in log p, T_{k+1} = b_k T_k (Sect. 2.5.1)."""
    lp = np.log10(p_bar)
    knots_lp = np.linspace(lp[0], lp[-1], len(b) + 1)
    knots_T = [T1]
    for bk in b:
        knots_T.append(knots_T[-1] * bk)
    # np.interp needs increasing x: log p decreases upward
    return np.interp(lp, knots_lp[::-1], np.array(knots_T)[::-1])


def log_uniform(rng, lo, hi, size=None):
    return 10.0 ** rng.uniform(np.log10(lo), np.log10(hi), size)


# ------------------------------------------------------------- observations


def snapped_edges(table: Table, window: Window, edges_cm):
    """Snap edges to window points (nearest; ties away from the start) and drop repeats."""
    first = table.nu0_cm + window.begin * table.dnu_cm
    step = window.stride * table.dnu_cm
    idx = np.floor((np.asarray(edges_cm) - first) / step + 0.5).astype(np.int64)
    idx = np.unique(np.clip(idx, 0, window.count - 1))
    return first + idx * step


def log_edges(lo, hi, n_bins):
    return np.exp(np.linspace(np.log(lo), np.log(hi), n_bins + 1))


# ---------------------------------------------------------- configurations
# C1: 1 absorber, 200 lines, 5 T x 5 log p, 2000 nu at 1 cm^-1, 20 layers,
#     isothermal + linear T(log p), 3 angles, R = 300, 50 bins.

C1_T = [300.0, 600.0, 900.0, 1200.0, 1500.0]
C1_LOGP = [-4.0, -2.5, -1.0, 0.5, 2.0]


def c1_table(seed=101):
    return make_table(seed, ["H2O"], C1_T, C1_LOGP, 4000.0, 1.0, 2000, n_lines=200,
                      s_range=(1e-23, 1e-19))


def c1_columns(seed=111):
    rng = np.random.default_rng(seed)
    p = levels(21, 2.0, -4.0)
    x = np.array([1e-3])
    cols = [Column(p, np.full(21, 900.0), x, 4.75, scale_factor(1.0)),
            Column(p, np.full(21, 1000.0), x, 4.75, scale_factor(1.0))]
    Tb = rng.uniform(1000.0, 1500.0)
    Tt = rng.uniform(300.0, Tb)
    cols.append(Column(p, linear_logp_profile(p, Tb, Tt), x, 4.75, scale_factor(1.0)))
    return cols


def c1_obs(table: Table):
    w = Window(0, table.n_nu, 1)
    return ObsSpec(w, 300.0, snapped_edges(table, w, log_edges(4050.0, 5950.0, 50)))


# C2: 8 absorbers + CIA, 27 T x 19 log p, 150k nu at 0.1 cm^-1 from 360,
#     100 layers (101 levels, 1e3 -> 1e-6 bar), 6-knot T(p), R = 300, 400 bins.

C2_SPECIES = ["H2O", "CH4", "CO", "CO2", "NH3", "H2S", "K", "X"]


def c2_table(seed=202, n_nu=150_000):
    return make_table(seed, C2_SPECIES, np.linspace(50.0, 3000.0, 27), np.linspace(-6.0, 3.0, 19),
                      360.0, 0.1, n_nu, n_lines=2000, bands=True, s_range=(1e-25, 1e-19),
                      with_cia=True)


def c2_like_column(rng, n_levels=101, n_species=8):
    p = levels(n_levels, 3.0, -6.0)
    T1 = rng.uniform(1500.0, 3000.0)
    b = rng.uniform(0.6, 0.95, 5)
    T = piecewise_knot_profile(p, T1, b)
    x = log_uniform(rng, 1e-8, 1e-2, n_species)
    return Column(p, T, x, float(rng.uniform(3.5, 6.0)), scale_factor(rng.uniform(0.1, 5.0)))


def c2_column(seed=212):
    return c2_like_column(np.random.default_rng(seed))


def c2_obs(table: Table):
    w = Window(0, table.n_nu, 1)
    return ObsSpec(w, 300.0, snapped_edges(table, w, log_edges(363.0, 15251.0, 400)))


# C3: the C1 grid with 512 sets from prior boxes.


def c3_columns(n_sets=512, seed=303):
    rng = np.random.default_rng(seed)
    p = levels(21, 2.0, -4.0)
    cols = []
    for _ in range(n_sets):
        Tb = rng.uniform(1000.0, 1500.0)
        b = rng.uniform(0.3, 0.95)
        cols.append(Column(p, linear_logp_profile(p, Tb, max(300.0, b * Tb)),
                           log_uniform(rng, 1e-8, 1e-2, 1), float(rng.uniform(3.5, 6.0)),
                           scale_factor(rng.uniform(0.1, 5.0))))
    return cols


# C4: the C2 batch (B sets) for reduced-precision tables.


def c4_columns(n_sets, seed=404, n_levels=101):
    rng = np.random.default_rng(seed)
    return [c2_like_column(rng, n_levels) for _ in range(n_sets)]


# C5: Poisson serving trace of uneven requests on the C2 table.


@dataclass
class TraceRequest:
    t_arrival: float
    obs: ObsSpec
    cols: List[Column]
    n_mu: int = 3


def c5_request(rng, table: Table, t_arrival=0.0, max_sets=64, span_range=(20_000, 150_000),
               strided_frac=0.5):
    layers = int(rng.integers(50, 201))
    span = int(rng.integers(span_range[0], min(span_range[1], table.n_nu) + 1))
    stride = 1 if rng.random() < 1.0 - strided_frac else 10
    begin = int(rng.integers(0, table.n_nu - span + 1))
    count = (span + stride - 1) // stride
    w = Window(begin, count, stride)
    R = float(rng.uniform(100.0, 1000.0))
    nu_first = table.nu0_cm + begin * table.dnu_cm
    nu_last = nu_first + (count - 1) * stride * table.dnu_cm
    c = 5.0 / (R * 2.0 * np.sqrt(2.0 * np.log(2.0)))
    lo = nu_first * (1.0 + c) + 2 * stride * table.dnu_cm
    hi = nu_last / (1.0 + c) - 2 * stride * table.dnu_cm
    if not hi > lo * (1.0 + 2.0 / R):
        # window narrower than the profile's margins: bins span the window
        lo = nu_first + 2 * stride * table.dnu_cm
        hi = nu_last - 2 * stride * table.dnu_cm
    n_bins = max(1, int(np.floor(R * np.log(hi / lo))))
    edges = snapped_edges(table, w, log_edges(lo, hi, n_bins))
    if len(edges) < 2:
        edges = snapped_edges(table, w, [nu_first, nu_last])
    n_sets = int(rng.integers(1, max_sets + 1))
    cols = [c2_like_column(rng, layers + 1, table.n_species) for _ in range(n_sets)]
    return TraceRequest(t_arrival, ObsSpec(w, R, edges), cols)


def c5_trace(table: Table, rate_hz=2000.0, duration_s=10.0, seed=505, max_requests=None,
             max_sets=64, span_range=(20_000, 150_000)):
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    while True:
        t += rng.exponential(1.0 / rate_hz)
        if t > duration_s or (max_requests is not None and len(out) >= max_requests):
            break
        out.append(c5_request(rng, table, t, max_sets=max_sets, span_range=span_range))
    return out


# Packed form of the serving trace (one array per column field), as a
# sampler hands its live points over.


@dataclass
class PackedRequest:
    t_arrival: float
    obs: ObsSpec
    p: np.ndarray       # [B][L]
    T: np.ndarray       # [B][L]
    x: np.ndarray       # [B][S]
    log_g: np.ndarray   # [B]
    scale: np.ndarray   # [B]
    n_mu: int = 3

    @property
    def n_sets(self) -> int:
        return int(self.p.shape[0])

    @property
    def layer_nu(self) -> int:
        return (self.p.shape[1] - 1) * self.obs.window.count * self.n_sets


def packed_c2_like_columns(rng, n_sets, n_levels, n_species):
    p = levels(n_levels, 3.0, -6.0)
    lp = np.log10(p)
    T1 = rng.uniform(1500.0, 3000.0, n_sets)
    b = rng.uniform(0.6, 0.95, (n_sets, 5))
    knots_T = np.concatenate([T1[:, None], T1[:, None] * np.cumprod(b, axis=1)], axis=1)
    knots_lp = np.linspace(lp[0], lp[-1], 6)
    # element index and weight of each level (knots decrease in log p)
    e = np.clip(np.searchsorted(-knots_lp, -lp, side="right") - 1, 0, 4)
    w = (lp - knots_lp[e]) / (knots_lp[e + 1] - knots_lp[e])
    T = knots_T[:, e] + w[None, :] * (knots_T[:, e + 1] - knots_T[:, e])
    x = log_uniform(rng, 1e-8, 1e-2, (n_sets, n_species))
    lg = rng.uniform(3.5, 6.0, n_sets)
    sc = np.array([scale_factor(f) for f in rng.uniform(0.1, 5.0, n_sets)])
    return np.tile(p, (n_sets, 1)), T, x, lg, sc


def c5_trace_packed(table: Table, rate_hz=2000.0, duration_s=10.0, seed=505, max_sets=64,
                    span_range=(20_000, 150_000), strided_frac=0.5):
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    while True:
        t += rng.exponential(1.0 / rate_hz)
        if t > duration_s:
            break
        r = c5_request(rng, table, t, max_sets=1, span_range=span_range,
                       strided_frac=strided_frac)
        n_sets = int(rng.integers(1, max_sets + 1))
        L = r.cols[0].n_levels
        p, T, x, lg, sc = packed_c2_like_columns(rng, n_sets, L, table.n_species)
        out.append(PackedRequest(t, r.obs, p, T, x, lg, sc))
    return out


# ------------------------------------------------- observed data for ln L


def noisy_data(model_bins, seed, noise_frac=0.2):
    """Synthetic observation of a model spectrum: D = model + sigma x N(0, 1)
    with sigma = noise_frac x the median |model| (the noise of the paper's
    synthetic retrieval tests, Sect. 4.1), and the same sigma as every bin's
    error bar.  Returns (D, sigma)."""
    m = np.asarray(model_bins, dtype=np.float64)
    rng = np.random.default_rng(seed)
    sigma = np.full(m.shape, noise_frac * float(np.median(np.abs(m))))
    return m + sigma * rng.standard_normal(m.shape), sigma


# ------------------------------------------ parameter vectors (Theta -> column)


@dataclass
class ParamLayout:
    """How a parameter vector maps onto a column (mirrors hr2_param_layout):
    n_elements elements of order `order` for the temperature, n_levels levels
    from log10_p_bottom to log10_p_top, the radius of Eq. 9, and for every
    table species the free ratio it copies (species_src, -1 = absent) times
    species_factor."""
    n_elements: int
    order: int
    n_levels: int
    log10_p_bottom: float
    log10_p_top: float
    radius_cm: float
    n_free: int
    with_eps: bool
    species_src: np.ndarray      # int32 [n_species]
    species_factor: np.ndarray   # float64 [n_species]
    with_cloud: bool = False     # theta carries (tau_c, p_top_bar, bottom_frac)


# solar Na/K number ratio from the photospheric abundances log eps(Na) = 6.24
# and log eps(K) = 5.03 (Asplund et al. 2009)
SOLAR_NA_K = 10.0 ** (6.24 - 5.03)


def c2_param_layout(n_elements=3, order=2, with_eps=True):
    """The paper's brown-dwarf set-up on the C2 table: seven free mixing
    ratios (H2O, CH4, CO, CO2, NH3, H2S, K; the eighth table species stands
    for Na, a fixed multiple of K), 101 levels from 1e3 to 1e-6 bar."""
    src = np.array([0, 1, 2, 3, 4, 5, 6, 6], dtype=np.int32)
    fac = np.array([1, 1, 1, 1, 1, 1, 1, SOLAR_NA_K], dtype=np.float64)
    return ParamLayout(n_elements, order, 101, 3.0, -6.0, R_JUP_CM, 7, with_eps, src, fac)


def c1_param_layout(n_elements=2, order=2, with_eps=False, n_levels=20):
    """One absorber (the C1 table), levels as the C1 columns."""
    return ParamLayout(n_elements, order, n_levels, 2.0, -4.0, R_JUP_CM, 1, with_eps,
                       np.array([0], dtype=np.int32), np.array([1.0]))


def draw_theta(layout: ParamLayout, n_sets, seed, log10_eps_range=(-30.0, -28.0)):
    """Parameter vectors [log g, f, d_pc, T1, b_1..b_{N_T-1}, x_free..., (cloud), (log10 eps)]
    from boxes inside the paper's priors (b kept in 0.6-0.95 and x in
    1e-8-1e-2 so that the temperatures stay on typical table grids and the
    filler gas stays positive)."""
    rng = np.random.default_rng(seed)
    NT = layout.n_elements * layout.order + 1
    rows = []
    for _ in range(n_sets):
        th = [rng.uniform(3.5, 6.0), rng.uniform(0.1, 5.0), rng.normal(10.0, 0.05),
              rng.uniform(1000.0, 3000.0)]
        th += list(rng.uniform(0.6, 0.95, NT - 1))
        th += list(log_uniform(rng, 1e-8, 1e-2, layout.n_free))
        if layout.with_cloud:
            # log-uniform draws (App. B states the priors' kind, not their ranges)
            th += [log_uniform(rng, 1e-2, 1e2), log_uniform(rng, 1e-3, 10.0),
                   log_uniform(rng, 1.5, 10.0)]
        if layout.with_eps:
            th.append(rng.uniform(*log10_eps_range))
        rows.append(th)
    return np.array(rows, dtype=np.float64)
