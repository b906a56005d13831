"""ctypes binding of libhr2 (include/hr2.h): argument marshalling only.

Every step of the forward model runs in the HIP kernels of libhr2.so; this
module converts numpy host arrays and torch device tensors into the C ABI's
plain pointers and sizes.  Device memory and streams come from PyTorch.
If the library is missing, loading fails loudly: there is no other path.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_double, c_int, c_int64, c_size_t, c_uint64, c_void_p
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# HR2_LIB_PATH: another build of the library (the sanitizer test's host-only one)
LIB_PATH = os.environ.get("HR2_LIB_PATH", os.path.join(HERE, "libhr2.so"))

OK, NOT_READY = 0, 1
E_INVALID_ARG, E_OUT_OF_RANGE, E_NO_MEMORY, E_DEVICE = -1, -2, -3, -4
E_NOT_FOUND, E_UNSUPPORTED, E_CANCELLED = -5, -6, -7
STATUS_NAMES = {0: "HR2_OK", 1: "HR2_NOT_READY", -1: "HR2_E_INVALID_ARG",
                -2: "HR2_E_OUT_OF_RANGE", -3: "HR2_E_NO_MEMORY", -4: "HR2_E_DEVICE",
                -5: "HR2_E_NOT_FOUND", -6: "HR2_E_UNSUPPORTED", -7: "HR2_E_CANCELLED"}
DTYPES = {"f32": 0, "f16": 1, "bf16": 2, "f64": 3}
OFFSET_MODES = {"row": 0, "species": 1}
REQ_PENDING, REQ_RUNNING, REQ_DONE, REQ_ERROR, REQ_CANCELLED = range(5)
(OPT_CHUNKS, OPT_NU_PER_LANE, OPT_TIMING, OPT_SOURCE, OPT_ROW_POLICY, OPT_TILE_PAIRS,
 OPT_TIMING_KERNELS) = range(7)

_DP = POINTER(c_double)


class HR2Error(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class TablesDesc(ctypes.Structure):
    _fields_ = [("n_species", c_int), ("n_T", c_int), ("n_p", c_int),
                ("T_K", _DP), ("log10_p_bar", _DP), ("nu0_cm", c_double), ("dnu_cm", c_double),
                ("n_nu", c_int64), ("log10_sigma", _DP), ("molar_mass", _DP), ("n_cia", c_int),
                ("log10_k_cia", _DP), ("he_h2_ratio", c_double), ("dtype", c_int),
                ("offset_mode", c_int)]


class ColumnC(ctypes.Structure):
    _fields_ = [("n_levels", c_int), ("p_bar", _DP), ("T_K", _DP), ("x", _DP),
                ("log_g_cgs", c_double), ("scale", c_double), ("tau_cloud", c_double),
                ("p_cloud_top_bar", c_double), ("cloud_bottom_frac", c_double)]


class WindowC(ctypes.Structure):
    _fields_ = [("nu_begin", c_int64), ("nu_count", c_int64), ("nu_stride", c_int64)]


class ParamLayoutC(ctypes.Structure):
    _fields_ = [("n_elements", c_int), ("order", c_int), ("n_levels", c_int),
                ("log10_p_bottom", c_double), ("log10_p_top", c_double), ("radius_cm", c_double),
                ("n_free", c_int), ("with_cloud", c_int), ("with_eps", c_int),
                ("species_src", POINTER(c_int)),
                ("species_factor", _DP)]


class RequestC(ctypes.Structure):
    _fields_ = [("window", WindowC), ("resolving_power", c_double), ("n_bins", c_int),
                ("bin_edges_cm", _DP), ("n_sets", c_int), ("cols", POINTER(ColumnC)),
                ("n_mu", c_int)]


class RequestInfo(ctypes.Structure):
    _fields_ = [("state", c_int), ("t_submit", c_double), ("t_admit", c_double),
                ("t_done", c_double), ("error", c_int), ("n_bins", c_int), ("n_sets", c_int)]


class ServeStats(ctypes.Structure):
    _fields_ = [("steps", c_uint64), ("requests_done", c_uint64), ("requests_failed", c_uint64),
                ("max_inflight", c_uint64), ("max_step_requests", c_uint64),
                ("peak_bytes", c_size_t)]


EXPORTS = [
    "hr2_ctx_create", "hr2_ctx_destroy", "hr2_last_error", "hr2_ctx_set_option",
    "hr2_tables_create", "hr2_tables_destroy", "hr2_opacity", "hr2_rt_emission",
    "hr2_obs_create", "hr2_obs_destroy", "hr2_obs_n_bins", "hr2_convolve_bin",
    "hr2_forward_batch", "hr2_forward_batch_dev", "hr2_serve_create", "hr2_serve_submit",
    "hr2_serve_poll", "hr2_serve_wait", "hr2_serve_destroy", "hr2_serve_debug_fail_next_step",
    "hr2_serve_get_stats", "hr2_ctx_collect_timing", "hr2_serve_submit_packed",
    "hr2_serve_debug_hold", "hr2_obs_set_data", "hr2_loglike_batch", "hr2_loglike_batch_dev",
    "hr2_params_create", "hr2_params_destroy", "hr2_params_n_theta", "hr2_params_unpack_dev",
    "hr2_forward_params_dev", "hr2_forward_batch_dev_noalloc",
]

_lib = None


def load() -> ctypes.CDLL:
    """Load libhr2.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -m paper_1910_01070_amd.build` (no fallback exists)")
    L = ctypes.CDLL(LIB_PATH)
    vp = c_void_p
    sig = {
        "hr2_ctx_create": ([c_int, POINTER(vp)], c_int),
        "hr2_ctx_destroy": ([vp], None),
        "hr2_last_error": ([], ctypes.c_char_p),
        "hr2_ctx_set_option": ([vp, c_int, c_int], c_int),
        "hr2_tables_create": ([vp, POINTER(TablesDesc), POINTER(vp)], c_int),
        "hr2_tables_destroy": ([vp], None),
        "hr2_opacity": ([vp, vp, POINTER(ColumnC), WindowC, vp, vp], c_int),
        "hr2_rt_emission": ([vp, vp, POINTER(ColumnC), WindowC, vp, c_int, vp, vp], c_int),
        "hr2_obs_create": ([vp, vp, WindowC, c_double, c_int, _DP, POINTER(vp)], c_int),
        "hr2_obs_destroy": ([vp], None),
        "hr2_obs_n_bins": ([vp], c_int),
        "hr2_convolve_bin": ([vp, vp, vp, c_double, vp, vp], c_int),
        "hr2_forward_batch": ([vp, vp, vp, c_int, POINTER(ColumnC), c_int, vp, vp, vp], c_int),
        "hr2_forward_batch_dev": ([vp, vp, vp, c_int, c_int, vp, vp, vp, vp, vp, vp, c_int, vp,
                                   vp, vp, vp], c_int),
        "hr2_serve_create": ([vp, vp, c_size_t, c_int, POINTER(vp)], c_int),
        "hr2_serve_submit": ([vp, POINTER(RequestC), POINTER(c_uint64)], c_int),
        "hr2_serve_poll": ([vp, c_uint64, vp, c_size_t, POINTER(RequestInfo)], c_int),
        "hr2_serve_wait": ([vp, c_uint64, c_double, vp, c_size_t, POINTER(RequestInfo)], c_int),
        "hr2_serve_destroy": ([vp], None),
        "hr2_serve_debug_fail_next_step": ([vp], c_int),
        "hr2_serve_get_stats": ([vp, POINTER(ServeStats)], c_int),
        "hr2_ctx_collect_timing": ([vp, POINTER(c_double), POINTER(c_int64)], c_int),
        "hr2_serve_submit_packed": ([vp, WindowC, c_double, c_int, _DP, c_int, c_int, _DP, _DP,
                                     _DP, _DP, _DP, c_int, POINTER(c_uint64)], c_int),
        "hr2_serve_debug_hold": ([vp, c_int], c_int),
        "hr2_obs_set_data": ([vp, _DP, _DP], c_int),
        "hr2_loglike_batch": ([vp, vp, vp, c_int, POINTER(ColumnC), c_int, _DP, vp, vp, vp],
                              c_int),
        "hr2_loglike_batch_dev": ([vp, vp, vp, c_int, c_int, vp, vp, vp, vp, vp, vp, vp, c_int,
                                   vp, vp, vp, vp], c_int),
        "hr2_params_create": ([vp, vp, POINTER(ParamLayoutC), POINTER(vp)], c_int),
        "hr2_params_destroy": ([vp], None),
        "hr2_params_n_theta": ([vp], c_int),
        "hr2_params_unpack_dev": ([vp, vp, c_int, vp, vp, vp, vp, vp, vp, vp, vp, vp], c_int),
        "hr2_forward_params_dev": ([vp, vp, vp, vp, c_int, vp, c_int, vp, vp, vp, vp], c_int),
        "hr2_forward_batch_dev_noalloc": ([vp, vp, vp, c_int, c_int, vp, vp, vp, vp, vp, vp,
                                           c_int, vp, vp, vp, vp], c_int),
    }
    for name, (args, res) in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = res
    _lib = L
    return L


def last_error() -> str:
    return (load().hr2_last_error() or b"").decode()


def _check(st: int):
    if st != OK:
        raise HR2Error(st, last_error())


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(_DP)


def _stream(stream) -> Optional[int]:
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _dev_ptr(t, dtype, numel: int, name: str) -> int:
    import torch
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous() or t.numel() < numel:
        raise ValueError(f"{name} must be contiguous with at least {numel} elements")
    return t.data_ptr()


class _Columns:
    """Keeps the numpy arrays of a list of columns alive while C reads them."""

    def __init__(self, cols):
        self.keep = []
        self.arr = (ColumnC * len(cols))()
        for i, c in enumerate(cols):
            p, T, x = _f64(c.p_bar), _f64(c.T_K), _f64(c.x)
            self.keep += [p, T, x]
            cl = getattr(c, "cloud", None)
            tau, ptop, frac = (0.0, 0.0, 0.0) if cl is None else (float(v) for v in cl)
            self.arr[i] = ColumnC(len(p), _ptr(p), _ptr(T), _ptr(x), float(c.log_g), float(c.scale),
                                  tau, ptop, frac)


def window_c(window) -> WindowC:
    return WindowC(int(window.begin), int(window.count), int(window.stride))


class Context:
    def __init__(self, device: int = 0):
        L = load()
        h = c_void_p()
        _check(L.hr2_ctx_create(int(device), ctypes.byref(h)))
        self.handle = h
        self.device = device

    def set_option(self, opt: int, value: int):
        _check(load().hr2_ctx_set_option(self.handle, int(opt), int(value)))

    def collect_timing(self):
        """(ms_levels, ms_column, ms_convolve_bin) summed, and the number of timed calls."""
        ms = (c_double * 3)()
        n = c_int64()
        _check(load().hr2_ctx_collect_timing(self.handle, ms, ctypes.byref(n)))
        return (ms[0], ms[1], ms[2]), n.value

    def close(self):
        if self.handle:
            load().hr2_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Tables:
    """Resident cross-section + CIA tables (duck-typed source table)."""

    def __init__(self, ctx: Context, table, dtype: str = "f32", offset: str = "row"):
        """offset: 'row' (one log2 offset per table row) or 'species'."""
        self.ctx = ctx
        self.dtype_name = dtype
        sig = _f64(table.log10_sigma)
        S, nT, nP, n_nu = sig.shape
        Tax, lp, mass = _f64(table.T_K), _f64(table.log10_p_bar), _f64(table.molar_mass)
        cia = None if table.log10_k_cia is None else _f64(table.log10_k_cia)
        d = TablesDesc(S, nT, nP, _ptr(Tax), _ptr(lp), float(table.nu0_cm), float(table.dnu_cm),
                       n_nu, _ptr(sig), _ptr(mass), 0 if cia is None else cia.shape[0],
                       _ptr(cia) if cia is not None else None, float(table.he_h2_ratio),
                       DTYPES[dtype], OFFSET_MODES[offset])
        h = c_void_p()
        _check(load().hr2_tables_create(ctx.handle, ctypes.byref(d), ctypes.byref(h)))
        self.handle = h
        self.n_species, self.n_nu = S, n_nu
        self.nu0_cm, self.dnu_cm = float(table.nu0_cm), float(table.dnu_cm)

    @property
    def real(self):
        import torch
        return torch.float64 if self.dtype_name == "f64" else torch.float32

    def close(self):
        if self.handle:
            load().hr2_tables_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Obs:
    """Observation layout: window, resolving power, bin edges (Eq. 17, binning)."""

    def __init__(self, ctx: Context, tables: Tables, window, resolving_power: float, edges_cm):
        self.ctx, self.tables, self.window = ctx, tables, window
        e = _f64(edges_cm)
        h = c_void_p()
        _check(load().hr2_obs_create(ctx.handle, tables.handle, window_c(window),
                                     float(resolving_power), len(e) - 1, _ptr(e),
                                     ctypes.byref(h)))
        self.handle = h
        self.n_bins = len(e) - 1

    def set_data(self, D, sigma):
        """Observed binned flux and its 1-sigma errors (host, n_bins each), for ln L."""
        D, sg = _f64(D), _f64(sigma)
        if D.shape != (self.n_bins,) or sg.shape != (self.n_bins,):
            raise ValueError("D and sigma need n_bins values each")
        _check(load().hr2_obs_set_data(self.handle, _ptr(D), _ptr(sg)))

    def close(self):
        if self.handle:
            load().hr2_obs_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def opacity(ctx: Context, tables: Tables, col, window, chi, stream=None):
    cols = _Columns([col])
    n = len(cols.keep[0]) * int(window.count)
    _check(load().hr2_opacity(ctx.handle, tables.handle, cols.arr, window_c(window),
                              _dev_ptr(chi, tables.real, n, "chi"), _stream(stream)))


def rt_emission(ctx: Context, tables: Tables, col, window, chi, n_mu: int, fplus, stream=None):
    cols = _Columns([col])
    L = len(cols.keep[0])
    _check(load().hr2_rt_emission(ctx.handle, tables.handle, cols.arr, window_c(window),
                                  _dev_ptr(chi, tables.real, L * int(window.count), "chi"),
                                  int(n_mu), _dev_ptr(fplus, tables.real, int(window.count),
                                                      "fplus"), _stream(stream)))


def convolve_bin(ctx: Context, obs: Obs, fplus, scale: float, bins, stream=None):
    real = obs.tables.real
    _check(load().hr2_convolve_bin(ctx.handle, obs.handle,
                                   _dev_ptr(fplus, real, int(obs.window.count), "fplus"),
                                   float(scale), _dev_ptr(bins, real, obs.n_bins, "bins"),
                                   _stream(stream)))


def forward_batch(ctx: Context, tables: Tables, obs: Obs, cols: Sequence, n_mu: int, bins,
                  fplus=None, stream=None):
    cc = _Columns(cols)
    B = len(cols)
    real = tables.real
    fp = None if fplus is None else _dev_ptr(fplus, real, B * int(obs.window.count), "fplus")
    _check(load().hr2_forward_batch(ctx.handle, tables.handle, obs.handle, B, cc.arr, int(n_mu),
                                    _dev_ptr(bins, real, B * obs.n_bins, "bins"), fp,
                                    _stream(stream)))


def forward_batch_dev(ctx: Context, tables: Tables, obs: Obs, p, T, x, log_g, scale, n_mu: int,
                      bins, fplus=None, status=None, stream=None, cloud=None):
    """Columns already in device memory: p, T [B][L], x [B][S], log_g, scale [B],
    cloud None or [B][3] (float64)."""
    import torch
    B, L = p.shape
    f64 = torch.float64
    real = tables.real
    fp = None if fplus is None else _dev_ptr(fplus, real, B * int(obs.window.count), "fplus")
    sp = None if status is None else _dev_ptr(status, torch.int32, B, "status")
    cp = None if cloud is None else _dev_ptr(cloud, f64, 3 * B, "cloud")
    _check(load().hr2_forward_batch_dev(
        ctx.handle, tables.handle, obs.handle, B, L, _dev_ptr(p, f64, B * L, "p"),
        _dev_ptr(T, f64, B * L, "T"), _dev_ptr(x, f64, B * tables.n_species, "x"),
        _dev_ptr(log_g, f64, B, "log_g"), _dev_ptr(scale, f64, B, "scale"), cp, int(n_mu),
        _dev_ptr(bins, real, B * obs.n_bins, "bins"), fp, sp, _stream(stream)))


def forward_batch_dev_noalloc(ctx: Context, tables: Tables, obs: Obs, p, T, x, log_g, scale,
                              n_mu: int, bins, fplus=None, status=None, stream=None, cloud=None):
    """forward_batch_dev with the library's scratch in its fixed device array
    (hr2_forward_batch_dev_noalloc): allocates no device memory."""
    import torch
    B, L = p.shape
    f64 = torch.float64
    real = tables.real
    fp = None if fplus is None else _dev_ptr(fplus, real, B * int(obs.window.count), "fplus")
    sp = None if status is None else _dev_ptr(status, torch.int32, B, "status")
    cp = None if cloud is None else _dev_ptr(cloud, f64, 3 * B, "cloud")
    _check(load().hr2_forward_batch_dev_noalloc(
        ctx.handle, tables.handle, obs.handle, B, L, _dev_ptr(p, f64, B * L, "p"),
        _dev_ptr(T, f64, B * L, "T"), _dev_ptr(x, f64, B * tables.n_species, "x"),
        _dev_ptr(log_g, f64, B, "log_g"), _dev_ptr(scale, f64, B, "scale"), cp, int(n_mu),
        _dev_ptr(bins, real, B * obs.n_bins, "bins"), fp, sp, _stream(stream)))


def loglike_batch(ctx: Context, tables: Tables, obs: Obs, cols: Sequence, n_mu: int, lnl,
                  log10_eps=None, bins=None, stream=None):
    """ln L per set (Eq. 19, or Eq. 22-23 with log10_eps) into device float64 lnl[B]."""
    import torch
    cc = _Columns(cols)
    B = len(cols)
    eps = None
    if log10_eps is not None:
        eps = _f64(log10_eps)
        if eps.shape != (B,):
            raise ValueError("log10_eps needs one value per set")
    bp = None if bins is None else _dev_ptr(bins, tables.real, B * obs.n_bins, "bins")
    _check(load().hr2_loglike_batch(ctx.handle, tables.handle, obs.handle, B, cc.arr, int(n_mu),
                                    None if eps is None else _ptr(eps),
                                    _dev_ptr(lnl, torch.float64, B, "lnl"), bp, _stream(stream)))


def loglike_batch_dev(ctx: Context, tables: Tables, obs: Obs, p, T, x, log_g, scale, n_mu: int,
                      lnl, log10_eps=None, bins=None, status=None, stream=None, cloud=None):
    """Device-resident float64 columns (as forward_batch_dev); log10_eps a device [B] or None."""
    import torch
    B, L = p.shape
    f64 = torch.float64
    ep = None if log10_eps is None else _dev_ptr(log10_eps, f64, B, "log10_eps")
    bp = None if bins is None else _dev_ptr(bins, tables.real, B * obs.n_bins, "bins")
    sp = None if status is None else _dev_ptr(status, torch.int32, B, "status")
    cp = None if cloud is None else _dev_ptr(cloud, f64, 3 * B, "cloud")
    _check(load().hr2_loglike_batch_dev(
        ctx.handle, tables.handle, obs.handle, B, L, _dev_ptr(p, f64, B * L, "p"),
        _dev_ptr(T, f64, B * L, "T"), _dev_ptr(x, f64, B * tables.n_species, "x"),
        _dev_ptr(log_g, f64, B, "log_g"), _dev_ptr(scale, f64, B, "scale"), cp, ep, int(n_mu),
        _dev_ptr(lnl, f64, B, "lnl"), bp, sp, _stream(stream)))


class Params:
    """Parameter-vector layout (finite-element temperature, free chemistry,
    Eq. 9 scale): duck-typed `layout` with the fields of hr2_param_layout."""

    def __init__(self, ctx: Context, tables: Tables, layout):
        self.ctx, self.tables = ctx, tables
        self._src = np.ascontiguousarray(layout.species_src, dtype=np.int32)
        self._fac = _f64(layout.species_factor)
        if self._src.shape != (tables.n_species,) or self._fac.shape != (tables.n_species,):
            raise ValueError("species_src and species_factor need one entry per table species")
        c = ParamLayoutC(int(layout.n_elements), int(layout.order), int(layout.n_levels),
                         float(layout.log10_p_bottom), float(layout.log10_p_top),
                         float(layout.radius_cm), int(layout.n_free),
                         int(bool(getattr(layout, "with_cloud", False))), int(bool(layout.with_eps)),
                         self._src.ctypes.data_as(POINTER(c_int)), _ptr(self._fac))
        h = c_void_p()
        _check(load().hr2_params_create(ctx.handle, tables.handle, ctypes.byref(c),
                                        ctypes.byref(h)))
        self.handle = h
        self.n_theta = load().hr2_params_n_theta(h)
        self.n_levels = int(layout.n_levels)

    def unpack(self, theta, p, T, x, log_g, scale, log10_eps=None, stream=None, cloud=None):
        import torch
        f64 = torch.float64
        B = theta.shape[0]
        L, S = self.n_levels, self.tables.n_species
        _check(load().hr2_params_unpack_dev(
            self.ctx.handle, self.handle, B, _dev_ptr(theta, f64, B * self.n_theta, "theta"),
            _dev_ptr(p, f64, B * L, "p"), _dev_ptr(T, f64, B * L, "T"),
            _dev_ptr(x, f64, B * S, "x"), _dev_ptr(log_g, f64, B, "log_g"),
            _dev_ptr(scale, f64, B, "scale"),
            None if cloud is None else _dev_ptr(cloud, f64, 3 * B, "cloud"),
            None if log10_eps is None else _dev_ptr(log10_eps, f64, B, "log10_eps"),
            _stream(stream)))

    def close(self):
        if self.handle:
            load().hr2_params_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def forward_params_dev(ctx: Context, tables: Tables, obs: Obs, params: Params, theta, n_mu: int,
                       bins=None, lnl=None, status=None, stream=None):
    """Device parameter vectors theta[B][n_theta] (float64) -> bins and/or ln L."""
    import torch
    B = theta.shape[0]
    f64 = torch.float64
    bp = None if bins is None else _dev_ptr(bins, tables.real, B * obs.n_bins, "bins")
    lp = None if lnl is None else _dev_ptr(lnl, f64, B, "lnl")
    sp = None if status is None else _dev_ptr(status, torch.int32, B, "status")
    _check(load().hr2_forward_params_dev(
        ctx.handle, tables.handle, obs.handle, params.handle, B,
        _dev_ptr(theta, f64, B * params.n_theta, "theta"), int(n_mu), bp, lp, sp,
        _stream(stream)))


class Server:
    """Continuous-batching server over resident tables (hr2_serve_*)."""

    def __init__(self, ctx: Context, tables: Tables, budget_bytes: int, max_slots: int = 64):
        h = c_void_p()
        _check(load().hr2_serve_create(ctx.handle, tables.handle, int(budget_bytes),
                                       int(max_slots), ctypes.byref(h)))
        self.handle = h
        self.tables = tables
        self.np_real = np.float64 if tables.dtype_name == "f64" else np.float32

    def submit(self, window, resolving_power: float, edges_cm, cols, n_mu: int = 3) -> int:
        cc = _Columns(cols)
        e = _f64(edges_cm)
        req = RequestC(window_c(window), float(resolving_power), len(e) - 1, _ptr(e), len(cols),
                       ctypes.cast(cc.arr, POINTER(ColumnC)), int(n_mu))
        t = c_uint64()
        _check(load().hr2_serve_submit(self.handle, ctypes.byref(req), ctypes.byref(t)))
        return t.value

    def submit_packed(self, window, resolving_power: float, edges_cm, p, T, x, log_g, scale,
                      n_mu: int = 3) -> int:
        """Columns as packed float64 arrays p, T [B][L], x [B][S], log_g, scale [B]."""
        e, p, T, x = _f64(edges_cm), _f64(p), _f64(T), _f64(x)
        lg, sc = _f64(log_g), _f64(scale)
        B, L = p.shape
        t = c_uint64()
        _check(load().hr2_serve_submit_packed(self.handle, window_c(window),
                                              float(resolving_power), len(e) - 1, _ptr(e), B, L,
                                              _ptr(p), _ptr(T), _ptr(x), _ptr(lg), _ptr(sc),
                                              int(n_mu), ctypes.byref(t)))
        return t.value

    def poll(self, ticket: int, n_elems: int, wait_s: Optional[float] = None):
        """Returns (status, results or None, info)."""
        out = np.empty(n_elems, dtype=self.np_real)
        info = RequestInfo()
        L = load()
        if wait_s is None:
            st = L.hr2_serve_poll(self.handle, int(ticket), out.ctypes.data_as(c_void_p), n_elems,
                                  ctypes.byref(info))
        else:
            st = L.hr2_serve_wait(self.handle, int(ticket), float(wait_s),
                                  out.ctypes.data_as(c_void_p), n_elems, ctypes.byref(info))
        return st, (out if st == OK else None), info

    def hold(self, on: bool):
        _check(load().hr2_serve_debug_hold(self.handle, 1 if on else 0))

    def fail_next_step(self):
        _check(load().hr2_serve_debug_fail_next_step(self.handle))

    def stats(self) -> ServeStats:
        s = ServeStats()
        _check(load().hr2_serve_get_stats(self.handle, ctypes.byref(s)))
        return s

    def close(self):
        if self.handle:
            load().hr2_serve_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
