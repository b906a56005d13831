"""CPU checks of the C ABI: the built library exports every function that
include/hr2.h declares, argument checks that need no device return the
documented codes, and the binding fails loudly when the library is missing."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_1910_01070_amd import hr2

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hr2.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(hr2_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ["hr2_opacity", "hr2_rt_emission", "hr2_convolve_bin", "hr2_forward_batch",
                     "hr2_serve_submit", "hr2_serve_poll"]:
        assert required in names


def test_library_exports_every_declared_symbol():
    lib = hr2.load()
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    assert set(hr2.EXPORTS) <= set(declared_functions())


def test_null_arguments_without_a_device():
    lib = hr2.load()
    out = ctypes.c_void_p()
    assert lib.hr2_ctx_create(0, None) == hr2.E_INVALID_ARG
    assert lib.hr2_tables_create(None, None, ctypes.byref(out)) == hr2.E_INVALID_ARG
    assert "NULL" in hr2.last_error()
    assert lib.hr2_serve_poll(None, 1, None, 0, None) == hr2.E_INVALID_ARG
    assert lib.hr2_serve_get_stats(None, None) == hr2.E_INVALID_ARG
    assert lib.hr2_obs_n_bins(None) == 0
    lib.hr2_ctx_destroy(None)
    lib.hr2_tables_destroy(None)
    lib.hr2_obs_destroy(None)
    lib.hr2_serve_destroy(None)
    assert lib.hr2_ctx_set_option(None, 0, 0) == hr2.E_INVALID_ARG
    ms = (ctypes.c_double * 3)()
    assert lib.hr2_ctx_collect_timing(None, ms, None) == hr2.E_INVALID_ARG
    assert lib.hr2_obs_set_data(None, None, None) == hr2.E_INVALID_ARG
    assert lib.hr2_loglike_batch(None, None, None, 1, None, 3, None, None, None,
                                 None) == hr2.E_INVALID_ARG
    assert lib.hr2_loglike_batch_dev(None, None, None, 1, 2, None, None, None, None, None, None,
                                     None, 3, None, None, None, None) == hr2.E_INVALID_ARG
    assert lib.hr2_forward_batch_dev_noalloc(None, None, None, 1, 2, None, None, None, None,
                                             None, None, 3, None, None, None,
                                             None) == hr2.E_INVALID_ARG
    assert lib.hr2_params_create(None, None, None, None) == hr2.E_INVALID_ARG
    assert lib.hr2_params_n_theta(None) == 0
    lib.hr2_params_destroy(None)
    assert lib.hr2_forward_params_dev(None, None, None, None, 1, None, 3, None, None, None,
                                      None) == hr2.E_INVALID_ARG


def test_context_without_a_device_reports_device_error():
    try:
        import torch
        if torch.cuda.is_available():
            pytest.skip("a device is present")
    except ImportError:
        pass
    lib = hr2.load()
    h = ctypes.c_void_p()
    assert lib.hr2_ctx_create(0, ctypes.byref(h)) == hr2.E_DEVICE
    assert h.value is None


def _no_device():
    try:
        import torch
        return not torch.cuda.is_available()
    except ImportError:
        return True


def _desc(n_T, n_p, n_nu, dtype, n_cia, keep):
    T_axis = np.linspace(100.0, 3000.0, n_T)
    lp = np.linspace(-6.0, 3.0, n_p)
    dummy = np.zeros(64)   # never read: the sizes are refused first
    mass = np.array([18.0])
    keep += [T_axis, lp, dummy, mass]
    dp = lambda a: a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    d = hr2.TablesDesc()
    d.n_species, d.n_T, d.n_p = 1, n_T, n_p
    d.T_K, d.log10_p_bar = dp(T_axis), dp(lp)
    d.nu0_cm, d.dnu_cm, d.n_nu = 100.0, 0.01, n_nu
    d.log10_sigma, d.molar_mass = dp(dummy), dp(mass)
    d.n_cia, d.log10_k_cia = n_cia, dp(dummy)
    d.he_h2_ratio, d.dtype = 0.17, hr2.DTYPES[dtype]
    return d


@pytest.mark.skipif(not _no_device(), reason="the refusal is checked where no device exists")
def test_table_blocks_past_4_gib_are_refused_before_any_device_work():
    """Rows are addressed by 32-bit byte offsets: a species block, and the two
    CIA pair blocks together (one buffer resource in the column kernel), must
    stay below 4 GiB.  The sizes are refused before the context is used or an
    array is read, so a stand-in context (zeroed memory) is enough here: if the
    check were missing, the call would go on to the device and fail with
    HR2_E_DEVICE instead."""
    lib = hr2.load()
    fake_ctx = ctypes.create_string_buffer(4096)
    out = ctypes.c_void_p()
    keep = []
    # one CIA pair block is 2.15 GB, both together 4.295e9 B >= 4 GiB; the
    # FP16 species block (256 x 2 rows) is 2.15 GB
    n_nu = (1 << 21) + 64
    d = _desc(256, 2, n_nu, "f16", 2, keep)
    assert lib.hr2_tables_create(fake_ctx, ctypes.byref(d), ctypes.byref(out)) == hr2.E_OUT_OF_RANGE
    assert "CIA" in hr2.last_error() and out.value is None
    # the same table without CIA gets past the size checks (and then needs a device)
    d = _desc(256, 2, n_nu, "f16", 0, keep)
    assert lib.hr2_tables_create(fake_ctx, ctypes.byref(d), ctypes.byref(out)) == hr2.E_DEVICE
    # an FP32 species block of 256 x 2 rows of that length is 4.295e9 B
    d = _desc(256, 2, n_nu, "f32", 0, keep)
    assert lib.hr2_tables_create(fake_ctx, ctypes.byref(d), ctypes.byref(out)) == hr2.E_OUT_OF_RANGE
    assert "species block" in hr2.last_error()
    # an unknown offset mode is refused before anything else
    d = _desc(4, 2, 64, "f16", 0, keep)
    d.offset_mode = 2
    assert lib.hr2_tables_create(fake_ctx, ctypes.byref(d), ctypes.byref(out)) == hr2.E_INVALID_ARG
    assert "offset_mode" in hr2.last_error()


def test_binding_fails_loudly_without_the_library(monkeypatch, tmp_path):
    monkeypatch.setattr(hr2, "_lib", None)
    monkeypatch.setattr(hr2, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(ImportError):
        hr2.load()


def test_struct_layouts_match_the_header():
    # sizes of the by-value / pointed-to structs on x86-64
    assert ctypes.sizeof(hr2.WindowC) == 24
    assert ctypes.sizeof(hr2.ColumnC) == 72
    assert ctypes.sizeof(hr2.TablesDesc) == 104
    assert hr2.TablesDesc.offset_mode.offset == 100
    assert ctypes.sizeof(hr2.ServeStats) == 48
    assert ctypes.sizeof(hr2.ParamLayoutC) == 72


def test_serving_trace_inputs_are_valid():
    import workloads as wl
    tab = wl.make_table(1, ["H2O", "CH4"], [300.0, 3000.0], [-6.0, 3.0], 360.0, 0.1, 150_000,
                        n_lines=5)
    rng = np.random.default_rng(0)
    for _ in range(50):
        r = wl.c5_request(rng, tab, 0.0, max_sets=3)
        e = r.obs.edges_cm
        assert len(e) >= 2 and np.all(np.diff(e) > 0)
        w = r.obs.window
        assert w.begin + (w.count - 1) * w.stride < tab.n_nu
        for c in r.cols:
            assert np.all(np.diff(c.p_bar) < 0) and np.all(c.T_K > 0) and c.x.sum() < 1
