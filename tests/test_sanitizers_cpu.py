"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only):
the FP64 oracle (plain C) and the host side of libhr2 (argument validation,
table limits, the C ABI checks of tests/test_abi_cpu.py) are rebuilt with the
sanitizers into a temporary directory and exercised in a child process with
the sanitizer runtime preloaded; any report fails the test.  The sanitizers
apply to host code only (-Xarch_host); nothing here touches a GPU."""
import os
import subprocess
import sys
import textwrap

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1910_01070_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
# host-only sanitizer flags: -Xarch_host in front of each, so no device code
# is ever built with them
SAN_HOST = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=undefined"]


def _run(cmd, env=None, timeout=600):
    p = subprocess.run(cmd, capture_output=True, text=True, env=env, timeout=timeout)
    return p.returncode, p.stdout + p.stderr


def _asan_runtime(compiler):
    rc, out = _run([compiler, "-print-file-name=" + ("libasan.so" if "gcc" in compiler
                                                     else "libclang_rt.asan-x86_64.so")])
    path = out.strip().splitlines()[-1] if rc == 0 and out.strip() else ""
    return path if os.path.isabs(path) and os.path.exists(path) else None


def _child_env(preload, **extra):
    env = dict(os.environ)
    env["LD_PRELOAD"] = preload
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=0:halt_on_error=1"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    env["PYTHONPATH"] = ROOT
    env.update(extra)
    return env


def _no_reports(out):
    return "ERROR: AddressSanitizer" not in out and "runtime error:" not in out


def test_oracle_under_asan_ubsan(tmp_path):
    rt = _asan_runtime("gcc")
    if rt is None:
        pytest.skip("gcc's AddressSanitizer runtime is not installed")
    lib = str(tmp_path / "liboracle_san.so")
    rc, out = _run(["gcc", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                    "-fno-sanitize-recover=undefined", "-fopenmp", "-fPIC", "-shared", "-o", lib,
                    os.path.join(ROOT, "oracle", "hr2_oracle.c"), "-lm"])
    assert rc == 0, out
    script = textwrap.dedent("""
        import numpy as np
        import oracle, workloads as wl
        from tests import hr2_testutil as tu
        assert oracle.LIB_PATH.endswith("liboracle_san.so"), oracle.LIB_PATH
        tab = tu.small_multi_table()
        col = tu.small_columns(tab, 1, seed=3)[0]
        w = wl.Window(7, 700, 3)
        nu0, dnu = oracle.window_grid(tab, w)
        edges = wl.snapped_edges(tab, w, wl.log_edges(nu0 + 60 * dnu, nu0 + 640 * dnu, 9))
        for order in (1, 2):
            r = oracle.forward(tab, col, w, 400.0, edges, 3, order=order)
            assert np.all(np.isfinite(r["bins"]))
        cloudy = wl.Column(col.p_bar, col.T_K, col.x, col.log_g, col.scale, (3.0, 0.01, 5.0))
        r = oracle.forward(tab, cloudy, w, 400.0, edges, 8, order=2)
        assert np.all(np.isfinite(r["bins"]))
        sub = oracle.forward_bins_subset(tab, col, w, 400.0, edges, 3, [0, 4, 8])
        fp = r["fplus"]
        a = oracle.convolve(fp, nu0, dnu, 400.0, banded=False)
        b = oracle.convolve(fp, nu0, dnu, 400.0, banded=True)
        assert np.allclose(a, b, rtol=1e-12)
        for n in range(1, 9):
            mu, wt = oracle.gauss_legendre01(n)
        print("lnl", oracle.log_likelihood(r["bins"], r["bins"] * 1.01, np.abs(r["bins"]) * 0.1,
                                          -3.0))
        print("oracle ok")
    """)
    rc, out = _run([sys.executable, "-c", script],
                   env=_child_env(rt, HR2_ORACLE_LIB=lib, OMP_NUM_THREADS="4"))
    assert rc == 0 and _no_reports(out) and "oracle ok" in out, out[-4000:]


def test_library_host_code_under_asan_ubsan(tmp_path):
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc is not installed")
    rt = _asan_runtime("/opt/rocm/llvm/bin/clang")
    if rt is None:
        pytest.skip("clang's AddressSanitizer runtime is not installed")
    # the device code is compiled unoptimised (it never runs here: there is
    # no GPU) only so that the objects link; the host code gets the sanitizers
    objs, procs = [], []
    for src in ("kernels.hip", "api.cpp", "serve.cpp", "noalloc.hip"):
        obj = str(tmp_path / (src + ".o"))
        opt = "-O0" if src.endswith(".hip") else "-O1"
        procs.append(subprocess.Popen(
            [HIPCC, "--offload-arch=gfx950", opt, "-g", "-std=c++17", "-fPIC", "-pthread",
             *SAN_HOST, "-I" + os.path.join(ROOT, "include"), "-I" + CSRC, "-c",
             os.path.join(CSRC, src), "-o", obj],
            stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True))
        objs.append(obj)
    for p in procs:
        out, _ = p.communicate(timeout=900)
        assert p.returncode == 0, out
    lib = str(tmp_path / "libhr2_san.so")
    rc, out = _run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-pthread", *SAN_HOST,
                    "-o", lib, *objs])
    assert rc == 0, out
    rc, out = _run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider",
                    os.path.join(ROOT, "tests", "test_abi_cpu.py")],
                   env=_child_env(rt, HR2_LIB_PATH=lib))
    assert rc == 0 and _no_reports(out), out[-4000:]
