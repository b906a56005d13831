"""A table larger than 4 GiB on the device (two species of 8 T x 8 log p rows
of 8.5 M wavenumbers, FP32: 4.35 GB): the column kernel then addresses each
species block through its own buffer resource, and the stage-1 kernel uses
64-bit species offsets.  A window at the far end of the table (byte offsets
past 4 GiB), FP32 against the FP64 oracle on the same window."""
import numpy as np
import pytest

import oracle
import workloads as wl
from tests import hr2_testutil as tu

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_1910_01070_amd import hr2  # noqa: E402


def say(*a):
    print(*a, flush=True)


def big_table():
    S, nT, nP, n_nu = 2, 8, 8, 8_500_000
    T = np.linspace(300.0, 2400.0, nT)
    lp = np.linspace(-4.0, 3.0, nP)
    nu0, dnu = 2000.0, 0.001
    k = np.arange(n_nu, dtype=np.float64)
    wave = np.sin(2.0 * np.pi * k / 3700.0) + 0.3 * np.sin(2.0 * np.pi * k / 251.0)
    sig = np.empty((S, nT, nP, n_nu), dtype=np.float64)
    for s in range(S):
        for t in range(nT):
            for p in range(nP):
                sig[s, t, p] = (-21.5 + 0.4 * s + 0.15 * t - 0.05 * p) + (0.6 + 0.1 * s) * wave
    return wl.Table(T_K=T, log10_p_bar=lp, nu0_cm=nu0, dnu_cm=dnu, n_nu=n_nu,
                    log10_sigma=sig, molar_mass=np.array([18.0, 16.0]), species=["A", "B"])


def test_table_over_4gib():
    assert torch.cuda.is_available()
    say("building the host table (8.7 GB FP64)")
    tab = big_table()
    ctx = hr2.Context(0)
    say("uploading (4.35 GB FP32)")
    T = hr2.Tables(ctx, tab, "f32")
    n = 3000
    w = wl.Window(tab.n_nu - n, n, 1)
    nu_first, dnu = oracle.window_grid(tab, w)
    edges = wl.snapped_edges(tab, w, wl.log_edges(nu_first + 0.2 * n * dnu,
                                                   nu_first + 0.8 * n * dnu, 5))
    obs = hr2.Obs(ctx, T, w, 2.0e6, edges)
    L = 21
    p = wl.levels(L, 2.5, -3.5)
    lev = np.arange(L)
    Tk = 1300.0 + 900.0 * np.sin(2.0 * np.pi * lev / 7.0)   # crosses T nodes both ways
    col = wl.Column(p, Tk, np.array([1e-3, 3e-4]), 4.5, wl.scale_factor(1.0))
    ref = oracle.forward(tab, col, w, 2.0e6, edges, 3)
    for chunks in (1, 3):
        ctx.set_option(hr2.OPT_CHUNKS, chunks)
        bins = torch.empty(obs.n_bins, dtype=torch.float32, device="cuda")
        fplus = torch.empty(n, dtype=torch.float32, device="cuda")
        hr2.forward_batch(ctx, T, obs, [col], 3, bins, fplus)
        torch.cuda.synchronize()
        e_f, _ = tu.max_rel_err(fplus.cpu().numpy().astype(np.float64), ref["fplus"])
        e_b, _ = tu.max_rel_err(bins.cpu().numpy().astype(np.float64), ref["bins"])
        say(f"  chunks {chunks}: F+ {e_f:.2e} bins {e_b:.2e}")
        assert e_f <= 1e-5 and e_b <= 1e-5
    ctx.set_option(hr2.OPT_CHUNKS, 0)
    say("stage 1 alone")
    chi = torch.empty(L * n, dtype=torch.float32, device="cuda")
    hr2.opacity(ctx, T, col, w, chi)
    torch.cuda.synchronize()
    chi_ref = oracle.opacity(tab, col, oracle.window_indices(w))
    e, _ = tu.max_rel_err(chi.cpu().numpy().astype(np.float64).reshape(L, n), chi_ref)
    say(f"  chi {e:.2e}")
    assert e <= 1e-5
    obs.close()
    T.close()
    ctx.close()
