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
