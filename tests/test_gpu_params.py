"""GPU parity of the parameter-vector path: hr2_params_unpack_dev against the
oracle's unpack (finite-element temperature, free chemistry, Eq. 9 scale),
and hr2_forward_params_dev (parameters -> bins and ln L) against the oracle's
forward model and likelihood on the oracle's own columns.

Tolerances: the unpacked columns agree to 1e-13 relative (FP64 both sides,
rounding order only); bins as the column path (1e-12 FP64 tables, 1e-5
FP32); ln L within the bound derived in test_gpu_likelihood from the bins'
tolerance."""
import numpy as np
import pytest

import oracle
from oracle import params as op
import workloads as wl
from tests import hr2_testutil as tu
from tests.test_gpu_likelihood import lnl_bound

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


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def oracle_column(lay, th):
    p, T, x, lg, sc, cloud, eps = op.unpack(lay, th)
    return wl.Column(p, T, x, lg, sc, cloud), eps


def rel(a, b):
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    return float(np.max(np.abs(a - b) / np.maximum(np.abs(b), 1e-300)))


@pytest.mark.parametrize("K,q", [(6, 1), (3, 2), (2, 4), (1, 8), (42, 3)])
def test_unpack_matches_oracle(ctx, K, q):
    c2_species = len(wl.C2_SPECIES)
    # a table with the C2 species list is only needed for its species count
    small = wl.make_table(5, wl.C2_SPECIES, [300.0, 3000.0], [-6.0, 3.0], 1000.0, 1.0, 256,
                          n_lines=20)
    T_ = hr2.Tables(ctx, small, "f64")
    lay = wl.c2_param_layout(K, q, with_eps=True)
    lay.n_levels = 70 if K != 42 else 1024
    P = hr2.Params(ctx, T_, lay)
    assert P.n_theta == op.n_theta(lay)
    th = wl.draw_theta(lay, 16, seed=K * 100 + q)
    if K == 42:
        th[:, 4:4 + K * q] = np.clip(th[:, 4:4 + K * q], 0.97, None)   # stay above ~1 K
    B, L, S = len(th), lay.n_levels, c2_species
    out = [torch.empty(B * n, dtype=torch.float64, device="cuda") for n in (L, L, S, 1, 1, 1)]
    say(f"unpack K={K} q={q} L={L}")
    P.unpack(dev(th), *out)
    torch.cuda.synchronize()
    p, T, x, lg, sc, eps = [o.cpu().numpy() for o in out]
    for s in range(B):
        rp, rT, rx, rlg, rsc, rcl, reps = op.unpack(lay, th[s])
        assert rel(p[s * L:(s + 1) * L], rp) <= 1e-13
        assert rel(T[s * L:(s + 1) * L], rT) <= 1e-13, (s, rel(T[s * L:(s + 1) * L], rT))
        assert np.array_equal(x[s * S:(s + 1) * S], rx)
        assert lg[s] == rlg and rel(sc[s], rsc) <= 1e-14 and eps[s] == reps
    P.close()
    T_.close()


@pytest.mark.parametrize("dtype,tol,tau", [("f64", 1e-12, 1e-12), ("f32", 1e-5, 1e-5)])
def test_c1_params_to_bins_and_lnl(ctx, dtype, tol, tau):
    tab = tu.c1_table()
    spec = wl.c1_obs(tab)
    lay = wl.c1_param_layout(2, 2, with_eps=True)
    T = hr2.Tables(ctx, tab, dtype)
    obs = hr2.Obs(ctx, T, spec.window, spec.resolving_power, spec.edges_cm)
    P = hr2.Params(ctx, T, lay)
    th = wl.draw_theta(lay, 6, seed=77)
    cols = [oracle_column(lay, t)[0] for t in th]
    refs = [oracle.forward(tab, c, spec.window, spec.resolving_power, spec.edges_cm, 3)["bins"]
            for c in cols]
    D, sigma = wl.noisy_data(refs[0], seed=123)
    obs.set_data(D, sigma)
    th[:, -1] = np.log10(float(sigma[0]) ** 2) + np.linspace(-1, 1, len(th))
    B = len(th)
    bins = torch.empty(B * obs.n_bins, dtype=T.real, device="cuda")
    lnl = torch.empty(B, dtype=torch.float64, device="cuda")
    status = torch.full((B,), 7, dtype=torch.int32, device="cuda")
    say(f"C1 {dtype}: parameters -> bins + ln L")
    hr2.forward_params_dev(ctx, T, obs, P, dev(th), 3, bins, lnl, status)
    torch.cuda.synchronize()
    b = bins.cpu().numpy().astype(np.float64).reshape(B, -1)
    ll = lnl.cpu().numpy()
    assert int(status.abs().sum()) == 0
    for s in range(B):
        e, _ = tu.max_rel_err(b[s], refs[s])
        want = oracle.log_likelihood(refs[s], D, sigma, th[s, -1])
        say(f"  set {s}: bins {e:.2e}  ln L diff {abs(ll[s] - want):.2e}")
        assert e <= tol
        assert abs(ll[s] - want) <= lnl_bound(refs[s], D, sigma, tau, th[s, -1])
    say("same as unpack + hr2_loglike_batch_dev")
    L, S = lay.n_levels, tab.n_species
    cols_d = [torch.empty(B * n, dtype=torch.float64, device="cuda") for n in (L, L, S, 1, 1, 1)]
    P.unpack(dev(th), *cols_d)
    lnl2 = torch.empty(B, dtype=torch.float64, device="cuda")
    bins2 = torch.empty_like(bins)
    p, Tk, x, lg, sc, eps = cols_d
    hr2.loglike_batch_dev(ctx, T, obs, p.view(B, L), Tk.view(B, L), x.view(B, S), lg, sc, 3, lnl2,
                          eps, bins2)
    torch.cuda.synchronize()
    assert torch.equal(bins, bins2) and torch.equal(lnl, lnl2)
    say("bins only, and one invalid vector")
    th_bad = th.copy()
    th_bad[2, 5] = -0.5                   # a negative b
    hr2.forward_params_dev(ctx, T, obs, P, dev(th_bad), 3, bins2, None, status)
    torch.cuda.synchronize()
    st = status.cpu().numpy()
    out = bins2.cpu().numpy().astype(np.float64).reshape(B, -1)
    assert st[2] == hr2.E_INVALID_ARG and np.all(np.delete(st, 2) == 0)
    assert np.all(np.isnan(out[2]))
    assert np.array_equal(np.delete(out, 2, axis=0), np.delete(b, 2, axis=0))
    P.close()
    obs.close()
    T.close()


def test_c2_params_lnl(ctx):
    """The paper's free-chemistry set-up (three second-order elements, seven
    free ratios, eps: 18 parameters) on the C2 table, FP32."""
    tab = tu.c2_table()
    spec = wl.c2_obs(tab)
    lay = wl.c2_param_layout(3, 2, with_eps=True)
    T = hr2.Tables(ctx, tab, "f32")
    obs = hr2.Obs(ctx, T, spec.window, spec.resolving_power, spec.edges_cm)
    P = hr2.Params(ctx, T, lay)
    assert P.n_theta == 18
    th = wl.draw_theta(lay, 2, seed=2020)
    say("C2 oracle spectra of two parameter vectors")
    refs = []
    for t in th:
        col, _ = oracle_column(lay, t)
        refs.append(oracle.forward(tab, col, spec.window, spec.resolving_power, spec.edges_cm,
                                   3)["bins"])
    D, sigma = wl.noisy_data(refs[0], seed=5)
    obs.set_data(D, sigma)
    th[:, -1] = np.log10(float(sigma[0]) ** 2) - 0.3
    lnl = torch.empty(2, dtype=torch.float64, device="cuda")
    bins = torch.empty(2 * obs.n_bins, dtype=torch.float32, device="cuda")
    hr2.forward_params_dev(ctx, T, obs, P, dev(th), 3, bins, lnl)
    torch.cuda.synchronize()
    b = bins.cpu().numpy().astype(np.float64).reshape(2, -1)
    for s in range(2):
        e, _ = tu.max_rel_err(b[s], refs[s])
        want = oracle.log_likelihood(refs[s], D, sigma, th[s, -1])
        got = float(lnl[s])
        say(f"  set {s}: bins {e:.2e}, ln L {got:.8e} vs {want:.8e}")
        assert e <= 1e-5
        assert abs(got - want) <= lnl_bound(refs[s], D, sigma, 1e-5, th[s, -1])
    say("64 vectors from the prior boxes: every ln L finite; the coldest against the oracle")
    thb = wl.draw_theta(lay, 64, seed=164)
    thb[:, -1] = th[0, -1]
    lnl = torch.empty(64, dtype=torch.float64, device="cuda")
    hr2.forward_params_dev(ctx, T, obs, P, dev(thb), 3, None, lnl)
    torch.cuda.synchronize()
    ll = lnl.cpu().numpy()
    assert np.all(np.isfinite(ll))
    t_top = [op.unpack(lay, t)[1][-1] for t in thb]
    s = int(np.argmin(t_top))
    col, _ = oracle_column(lay, thb[s])
    ref = oracle.forward(tab, col, spec.window, spec.resolving_power, spec.edges_cm, 3)["bins"]
    want = oracle.log_likelihood(ref, D, sigma, thb[s, -1])
    say(f"  coldest top {t_top[s]:.0f} K: ln L {ll[s]:.8e} vs {want:.8e}")
    assert abs(ll[s] - want) <= lnl_bound(ref, D, sigma, 1e-5, thb[s, -1])
    P.close()
    obs.close()
    T.close()


def test_params_to_lnl_graph_replay(ctx):
    """hr2_forward_params_dev with ln L, captured once into a HIP graph after an
    eager call, replayed with eager work and synchronisations in between, with
    new parameter vectors copied in between replays: every replay equals an
    eager call on the same vectors."""
    tab = tu.c1_table()
    spec = wl.c1_obs(tab)
    lay = wl.c1_param_layout(2, 2, with_eps=True)
    T = hr2.Tables(ctx, tab, "f32")
    obs = hr2.Obs(ctx, T, spec.window, spec.resolving_power, spec.edges_cm)
    P = hr2.Params(ctx, T, lay)
    B = 64
    th_all = [wl.draw_theta(lay, B, seed=900 + r) for r in range(3)]
    ref0 = oracle.forward(tab, oracle_column(lay, th_all[0][0])[0], spec.window,
                          spec.resolving_power, spec.edges_cm, 3)["bins"]
    D, sigma = wl.noisy_data(ref0, seed=4)
    obs.set_data(D, sigma)
    for th in th_all:
        th[:, -1] = np.log10(float(sigma[0]) ** 2)
    theta = dev(th_all[0])
    bins = torch.empty(B * obs.n_bins, dtype=torch.float32, device="cuda")
    lnl = torch.empty(B, dtype=torch.float64, device="cuda")
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        hr2.forward_params_dev(ctx, T, obs, P, theta, 3, bins, lnl, None, s)
        s.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=s):
            hr2.forward_params_dev(ctx, T, obs, P, theta, 3, bins, lnl, None, s)
    torch.cuda.synchronize()
    for rep, th in enumerate(th_all):
        say(f"replay {rep}")
        theta.copy_(dev(th))
        want_l = torch.empty_like(lnl)
        want_b = torch.empty_like(bins)
        hr2.forward_params_dev(ctx, T, obs, P, theta, 3, want_b, want_l)
        torch.cuda.synchronize()
        bins.zero_()
        lnl.zero_()
        junk = torch.randn(1 << 16, device="cuda").sum()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(bins, want_b) and torch.equal(lnl, want_l), rep
        del junk
    del g
    torch.cuda.synchronize()
    P.close()
    obs.close()
    T.close()
