"""GPU parity of the fused likelihood (Eq. 19; error inflation Eq. 22-23).

Tolerance, derived from the model's: if every model bin m_j carries a
relative error of at most tau (1e-12 with FP64 tables, 1e-5 with FP32), the
residual r_j = D_j - m_j moves by d_j <= tau |m_j|, and the term
-r_j^2 / (2 s_j^2) by at most (|r_j| d_j + d_j^2 / 2) / s_j^2.  Summed over
the bins this bounds |ln L_gpu - ln L_oracle| (plus FP64 rounding of the
sum).  Separately, the likelihood arithmetic itself is checked tightly:
the oracle's ln L of the model bins the library returns must equal the
fused value to FP64 rounding."""
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


@pytest.fixture(scope="module")
def ctx():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    c = hr2.Context(0)
    yield c
    torch.cuda.synchronize()
    c.close()


def lnl_bound(model, D, sigma, tau, log10_eps=None):
    s2 = sigma ** 2 + (0.0 if log10_eps is None else 10.0 ** log10_eps)
    d = tau * np.abs(model)
    terms = -(D - model) ** 2 / (2 * s2) - 0.5 * np.log(2 * np.pi * s2)
    return (float(np.sum((np.abs(D - model) * d + 0.5 * d * d) / s2))
            + 1e-13 * float(np.sum(np.abs(terms))))


def fused(ctx, T, obs, cols, n_mu, eps=None):
    B = len(cols)
    lnl = torch.full((B,), 7.0, dtype=torch.float64, device="cuda")
    bins = torch.empty(B * obs.n_bins, dtype=T.real, device="cuda")
    hr2.loglike_batch(ctx, T, obs, cols, n_mu, lnl, eps, bins)
    torch.cuda.synchronize()
    return lnl.cpu().numpy(), bins.cpu().numpy().astype(np.float64).reshape(B, obs.n_bins)


@pytest.mark.parametrize("dtype,tau", [("f64", 1e-12), ("f32", 1e-5)])
def test_c1_loglike_matches_oracle(ctx, dtype, tau):
    tab = tu.c1_table()
    cols = wl.c1_columns()
    spec = wl.c1_obs(tab)
    T = hr2.Tables(ctx, tab, dtype)
    obs = hr2.Obs(ctx, T, spec.window, spec.resolving_power, spec.edges_cm)
    ref = [oracle.forward(tab, c, spec.window, spec.resolving_power, spec.edges_cm, 3)["bins"]
           for c in cols]
    D, sigma = wl.noisy_data(ref[0], seed=19)
    obs.set_data(D, sigma)
    eps = np.linspace(-1.0, 1.0, len(cols)) + np.log10(float(np.median(sigma)) ** 2)
    for use_eps in (False, True):
        e = eps if use_eps else None
        say(f"C1 {dtype}: ln L of {len(cols)} sets, inflation={use_eps}")
        lnl, bins = fused(ctx, T, obs, cols, 3, e)
        for s in range(len(cols)):
            es = None if e is None else float(e[s])
            want = oracle.log_likelihood(ref[s], D, sigma, es)
            bound = lnl_bound(ref[s], D, sigma, tau, es)
            say(f"  set {s}: ln L {lnl[s]:.10e} oracle {want:.10e} |diff| {abs(lnl[s] - want):.2e}"
                f" bound {bound:.2e}")
            assert abs(lnl[s] - want) <= bound
            same = oracle.log_likelihood(bins[s], D, sigma, es)
            assert abs(lnl[s] - same) <= 1e-12 * max(1.0, abs(same))
    obs.close()
    T.close()


def test_bins_and_repeatability(ctx):
    """The fused call's bins equal hr2_forward_batch's; repeated calls and a
    set alone give identical ln L (fixed-order reduction, independent sets)."""
    tab = tu.small_multi_table()
    cols = tu.small_columns(tab, 9)
    w = wl.Window(0, tab.n_nu, 1)
    nu = tab.nu0_cm + tab.dnu_cm * np.arange(tab.n_nu)
    edges = wl.log_edges(nu[40], nu[-40], 37)
    T = hr2.Tables(ctx, tab, "f32")
    obs = hr2.Obs(ctx, T, w, 400.0, edges)
    ref = oracle.forward(tab, cols[0], w, 400.0, edges, 4)["bins"]
    D, sigma = wl.noisy_data(ref, seed=3)
    obs.set_data(D, sigma)
    ctx.set_option(hr2.OPT_CHUNKS, 2)
    lnl, bins = fused(ctx, T, obs, cols, 4)
    fb = torch.empty(len(cols) * obs.n_bins, dtype=torch.float32, device="cuda")
    hr2.forward_batch(ctx, T, obs, cols, 4, fb)
    torch.cuda.synchronize()
    assert np.array_equal(fb.cpu().numpy().astype(np.float64).reshape(len(cols), -1), bins)
    lnl2, _ = fused(ctx, T, obs, cols, 4)
    assert np.array_equal(lnl, lnl2)
    one, _ = fused(ctx, T, obs, [cols[4]], 4)
    assert one[0] == lnl[4]
    want = oracle.log_likelihood(ref, D, sigma)
    assert abs(lnl[0] - want) <= lnl_bound(ref, D, sigma, 1e-5)
    say("bins only on request: lnl without bins")
    out = torch.empty(len(cols), dtype=torch.float64, device="cuda")
    hr2.loglike_batch(ctx, T, obs, cols, 4, out)
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy(), lnl)
    ctx.set_option(hr2.OPT_CHUNKS, 0)
    obs.close()
    T.close()


def test_device_entry_invalid_set_and_errors(ctx):
    tab = tu.c1_table()
    spec = wl.c1_obs(tab)
    T = hr2.Tables(ctx, tab, "f32")
    obs = hr2.Obs(ctx, T, spec.window, spec.resolving_power, spec.edges_cm)
    cols = wl.c3_columns(32, seed=21)
    B = len(cols)
    lnl = torch.empty(B, dtype=torch.float64, device="cuda")
    say("no data yet")
    with pytest.raises(hr2.HR2Error) as ei:
        hr2.loglike_batch(ctx, T, obs, cols, 3, lnl)
    assert ei.value.status == hr2.E_INVALID_ARG
    ref = oracle.forward(tab, cols[0], spec.window, spec.resolving_power, spec.edges_cm, 3)["bins"]
    D, sigma = wl.noisy_data(ref, seed=8)
    bad = sigma.copy()
    bad[3] = 0.0
    with pytest.raises(hr2.HR2Error):
        obs.set_data(D, bad)
    obs.set_data(D, sigma)
    with pytest.raises(hr2.HR2Error):
        hr2.loglike_batch(ctx, T, obs, cols, 3, lnl, np.full(B, np.inf))
    eps = np.full(B, np.log10(float(sigma[0]) ** 2))
    lnl_h, _ = fused(ctx, T, obs, cols, 3, eps)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()
    p = dev(np.stack([c.p_bar for c in cols]))
    Tk = dev(np.stack([c.T_K for c in cols]))
    x = dev(np.stack([c.x for c in cols]))
    lg = dev([c.log_g for c in cols])
    sc = dev([c.scale for c in cols])
    status = torch.full((B,), 7, dtype=torch.int32, device="cuda")
    say("device entry equals the host entry")
    hr2.loglike_batch_dev(ctx, T, obs, p, Tk, x, lg, sc, 3, lnl, dev(eps), None, status)
    torch.cuda.synchronize()
    assert np.array_equal(lnl.cpu().numpy(), lnl_h)
    assert int(status.abs().sum()) == 0
    say("one invalid set")
    Tbad = Tk.clone()
    Tbad[6, 2] = -1.0
    hr2.loglike_batch_dev(ctx, T, obs, p, Tbad, x, lg, sc, 3, lnl, dev(eps), None, status)
    torch.cuda.synchronize()
    got, st = lnl.cpu().numpy(), status.cpu().numpy()
    assert np.isnan(got[6]) and st[6] == hr2.E_INVALID_ARG
    assert np.array_equal(np.delete(got, 6), np.delete(lnl_h, 6))
    obs.close()
    T.close()


def test_c2_loglike(ctx):
    """C2 size (150000 points, 101 levels, 8 species, 400 bins), FP32, against
    the oracle's whole spectrum with 20%-of-median noise."""
    tab = tu.c2_table()
    spec = wl.c2_obs(tab)
    col = wl.c2_column()
    say("C2 oracle spectrum")
    ref = oracle.forward(tab, col, spec.window, spec.resolving_power, spec.edges_cm, 3)["bins"]
    D, sigma = wl.noisy_data(ref, seed=2019)
    T = hr2.Tables(ctx, tab, "f32")
    obs = hr2.Obs(ctx, T, spec.window, spec.resolving_power, spec.edges_cm)
    obs.set_data(D, sigma)
    for e in (None, np.array([np.log10(float(sigma[0]) ** 2) - 0.5])):
        lnl, bins = fused(ctx, T, obs, [col], 3, e)
        es = None if e is None else float(e[0])
        want = oracle.log_likelihood(ref, D, sigma, es)
        bound = lnl_bound(ref, D, sigma, 1e-5, es)
        say(f"  ln L {lnl[0]:.10e} oracle {want:.10e} |diff| {abs(lnl[0] - want):.2e} "
            f"bound {bound:.2e}")
        assert abs(lnl[0] - want) <= bound
        assert abs(lnl[0] - oracle.log_likelihood(bins[0], D, sigma, es)) <= 1e-12 * abs(want)
    obs.close()
    T.close()
