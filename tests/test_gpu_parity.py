"""GPU parity: the HIP path against the FP64 oracle on the same seeded inputs.

Tolerances (per spectrum, max relative error with a 1e-30 * max floor):
FP64 tables -> 1e-12, FP32 tables -> 1e-5 (F+ and bins), FP16 tables ->
1e-5 against the oracle on the dequantised table.  Every call goes through
the C ABI (ctypes binding)."""
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


def run_forward(ctx, tables, obs, cols, n_mu=3, chunks=0):
    ctx.set_option(hr2.OPT_CHUNKS, chunks)
    B = len(cols)
    bins = torch.empty(B * obs.n_bins, dtype=tables.real, device="cuda")
    fplus = torch.empty(B * obs.window.count, dtype=tables.real, device="cuda")
    hr2.forward_batch(ctx, tables, obs, cols, n_mu, bins, fplus)
    torch.cuda.synchronize()
    return (bins.cpu().numpy().reshape(B, obs.n_bins).astype(np.float64),
            fplus.cpu().numpy().reshape(B, obs.window.count).astype(np.float64))


# ------------------------------------------------------------------- C1


@pytest.mark.parametrize("dtype,tol", [("f64", 1e-12), ("f32", 1e-5)])
def test_c1_full_chain(ctx, dtype, tol):
    """C1: 1 absorber, 5x5 table, 2000 points, 20 layers, 3 angles, R=300, 50 bins."""
    tab = tu.c1_table()
    cols = wl.c1_columns()
    spec = wl.c1_obs(tab)
    say(f"C1 {dtype}: tables + layout")
    T = hr2.Tables(ctx, tab, dtype)
    obs = hr2.Obs(ctx, T, spec.window, spec.resolving_power, spec.edges_cm)
    for chunks in (0, 1, 2, 3, 4, 8):
        say(f"C1 {dtype}: forward, chunks={chunks}")
        bins, fplus = run_forward(ctx, T, obs, cols, 3, chunks)
        for s, col in enumerate(cols):
            ref = oracle.forward(tab, col, spec.window, spec.resolving_power, spec.edges_cm, 3)
            e_f, _ = tu.max_rel_err(fplus[s], ref["fplus"])
            e_b, _ = tu.max_rel_err(bins[s], ref["bins"])
            say(f"  set {s}: F+ {e_f:.2e} bins {e_b:.2e}")
            assert e_f <= tol and e_b <= tol, (dtype, chunks, s, e_f, e_b)


@pytest.mark.parametrize("dtype,tol", [("f64", 1e-12), ("f32", 1e-5)])
def test_angle_counts(ctx, dtype, tol):
    """The fused path at every angle count across the two compiled angle
    tiers (up to 3, and 4 to 8 angles), with one and with several layer
    chunks."""
    tab = tu.c1_table()
    cols = wl.c1_columns()[:2]
    spec = wl.c1_obs(tab)
    T = hr2.Tables(ctx, tab, dtype)
    obs = hr2.Obs(ctx, T, spec.window, spec.resolving_power, spec.edges_cm)
    for n_mu in (1, 2, 3, 4, 6, 8):
        refs = [oracle.forward(tab, c, spec.window, spec.resolving_power, spec.edges_cm, n_mu)
                for c in cols]
        for chunks in (1, 3):
            say(f"C1 {dtype}: n_mu={n_mu} chunks={chunks}")
            bins, fplus = run_forward(ctx, T, obs, cols, n_mu, chunks)
            for s, ref in enumerate(refs):
                e_f, _ = tu.max_rel_err(fplus[s], ref["fplus"])
                e_b, _ = tu.max_rel_err(bins[s], ref["bins"])
                assert e_f <= tol and e_b <= tol, (dtype, n_mu, chunks, s, e_f, e_b)
    obs.close()
    T.close()


@pytest.mark.parametrize("dtype,tol", [("f64", 1e-12), ("f32", 1e-5)])
def test_stage_calls(ctx, dtype, tol):
    """hr2_opacity, hr2_rt_emission and hr2_convolve_bin one at a time, each
    fed the oracle's previous stage."""
    tab = tu.small_multi_table()
    col = tu.small_columns(tab, 1, seed=3)[0]
    w = wl.Window(7, 2900, 1)
    T = hr2.Tables(ctx, tab, dtype)
    L = col.n_levels
    say(f"stage calls {dtype}: opacity")
    chi = torch.empty(L * w.count, dtype=T.real, device="cuda")
    hr2.opacity(ctx, T, col, w, chi)
    torch.cuda.synchronize()
    chi_ref = oracle.opacity(tab, col, oracle.window_indices(w))
    e, _ = tu.max_rel_err(chi.cpu().numpy().reshape(L, w.count), chi_ref)
    say(f"  chi {e:.2e}")
    assert e <= tol
    say(f"stage calls {dtype}: rt_emission from the oracle's chi")
    chi_in = torch.from_numpy(chi_ref.astype(np.float64 if dtype == "f64" else np.float32)).cuda()
    fplus = torch.empty(w.count, dtype=T.real, device="cuda")
    st = oracle.column_state(tab, col)
    nu = tab.nu0_cm + oracle.window_indices(w) * tab.dnu_cm
    for n_mu in (1, 2, 3, 4, 5, 8):
        ref = oracle.rt_emission(chi_ref, st["dz"], col.T_K, nu, n_mu)
        # automatic, upward only, and alternating upward / downward chunks
        for chunks in (0, 1, 2, 5):
            ctx.set_option(hr2.OPT_CHUNKS, chunks)
            hr2.rt_emission(ctx, T, col, w, chi_in.reshape(-1), n_mu, fplus)
            torch.cuda.synchronize()
            ctx.set_option(hr2.OPT_CHUNKS, 0)
            e, _ = tu.max_rel_err(fplus.cpu().numpy(), ref)
            say(f"  n_mu={n_mu} chunks={chunks}: F+ {e:.2e}")
            assert e <= tol, (n_mu, chunks, e)
    say(f"stage calls {dtype}: convolve_bin from the oracle's F+")
    edges = wl.snapped_edges(tab, w, wl.log_edges(2030.0, 3430.0, 37))
    obs = hr2.Obs(ctx, T, w, 250.0, edges)
    ref_f = oracle.rt_emission(chi_ref, oracle.column_state(tab, col)["dz"], col.T_K,
                               tab.nu0_cm + oracle.window_indices(w) * tab.dnu_cm, 3)
    fin = torch.from_numpy(ref_f.astype(np.float64 if dtype == "f64" else np.float32)).cuda()
    bins = torch.empty(obs.n_bins, dtype=T.real, device="cuda")
    hr2.convolve_bin(ctx, obs, fin, col.scale, bins)
    torch.cuda.synchronize()
    nu_first, dnu = oracle.window_grid(tab, w)
    idx = oracle.snap_edges(edges, nu_first, dnu, w.count)
    fd = np.zeros(w.count)
    fd[idx[0]:idx[-1] + 1] = oracle.convolve(ref_f, nu_first, dnu, 250.0,
                                             np.arange(idx[0], idx[-1] + 1))
    ref_b = oracle.bin_spectrum(fd, idx, nu_first, dnu, col.scale)
    e, _ = tu.max_rel_err(bins.cpu().numpy(), ref_b)
    say(f"  bins {e:.2e}")
    assert e <= tol


@pytest.mark.parametrize("dtype,tol", [("f64", 1e-12), ("f32", 1e-5)])
def test_multispecies_cia_windows(ctx, dtype, tol):
    """3 species + CIA; ragged and strided windows; L = 2 and L = 41; all chunkings."""
    tab = tu.small_multi_table()
    T = hr2.Tables(ctx, tab, dtype)
    cases = [(wl.Window(0, 3000, 1), 41), (wl.Window(13, 1001, 2), 41), (wl.Window(5, 333, 7), 41),
             (wl.Window(100, 2500, 1), 2), (wl.Window(0, 64, 1), 3)]
    for w, L in cases:
        cols = tu.small_columns(tab, 3, seed=L + w.begin, n_levels=L)
        nu_first, dnu = oracle.window_grid(tab, w)
        lo = nu_first + 0.2 * (w.count - 1) * dnu
        hi = nu_first + 0.8 * (w.count - 1) * dnu
        edges = wl.snapped_edges(tab, w, wl.log_edges(lo, hi, 9))
        obs = hr2.Obs(ctx, T, w, 400.0, edges)
        for chunks in (1, 2, 3, 5, 8):
            say(f"window {w} L={L} {dtype} chunks={chunks}")
            bins, fplus = run_forward(ctx, T, obs, cols, 3, chunks)
            for s, col in enumerate(cols):
                ref = oracle.forward(tab, col, w, 400.0, edges, 3)
                e_f, _ = tu.max_rel_err(fplus[s], ref["fplus"])
                e_b, _ = tu.max_rel_err(bins[s], ref["bins"])
                assert e_f <= tol and e_b <= tol, (w, L, chunks, s, e_f, e_b)


@pytest.mark.parametrize("dtype,tol", [("f64", 1e-12), ("f32", 1e-5), ("f16", None)])
def test_species_counts(ctx, dtype, tol):
    """Every compiled species variant of the column kernel: 2, 5 and 8 species
    (up to eight slots with guards, or exactly eight), 10 and 12 (the twelve-slot
    variant), with CIA, fused path and the stage-1 call, FP64/FP32 against the
    oracle and FP16 against the oracle on the dequantised table."""
    names = ["H2O", "CH4", "CO", "CO2", "NH3", "H2S", "K", "X", "Na", "TiO", "VO", "FeH"]
    for S in (2, 5, 8, 10, 12):
        tab = wl.make_table(600 + S, names[:S], [250.0, 700.0, 1400.0, 2300.0],
                            [-4.0, -1.5, 1.0, 2.5], 3000.0, 0.5, 700, n_lines=40,
                            with_cia=True)
        T = hr2.Tables(ctx, tab, dtype)
        ref_tab = tu.dequantised(tab, dtype) if dtype == "f16" else tab
        w = wl.Window(11, 650, 1)
        nu_first, dnu = oracle.window_grid(tab, w)
        edges = wl.snapped_edges(tab, w, wl.log_edges(nu_first + 60 * dnu, nu_first + 590 * dnu, 6))
        obs = hr2.Obs(ctx, T, w, 500.0, edges)
        cols = tu.small_columns(tab, 2, seed=S, n_levels=23)
        t = tol if tol is not None else 1e-5
        for chunks in (1, 3):
            say(f"{S} species {dtype} chunks={chunks}")
            bins, fplus = run_forward(ctx, T, obs, cols, 3, chunks)
            for s, col in enumerate(cols):
                ref = oracle.forward(ref_tab, col, w, 500.0, edges, 3)
                e_f, _ = tu.max_rel_err(fplus[s], ref["fplus"])
                e_b, _ = tu.max_rel_err(bins[s], ref["bins"])
                assert e_f <= t and e_b <= t, (S, dtype, chunks, s, e_f, e_b)
        chi = torch.empty(23 * w.count, dtype=T.real, device="cuda")
        hr2.opacity(ctx, T, cols[0], w, chi)
        torch.cuda.synchronize()
        chi_ref = oracle.opacity(ref_tab, cols[0], oracle.window_indices(w))
        e, _ = tu.max_rel_err(chi.cpu().numpy().astype(np.float64).reshape(23, -1), chi_ref)
        assert e <= t, (S, dtype, e)
        obs.close()
        T.close()


@pytest.mark.parametrize("dtype,tol", [("f64", 1e-12), ("f32", 1e-5)])
def test_most_levels(ctx, dtype, tol):
    """The largest column the library takes (HR2_MAX_LEVELS = 1024 levels) in
    one chunk, in the automatic chunking and in eight chunks."""
    tab = tu.small_multi_table()
    T = hr2.Tables(ctx, tab, dtype)
    w = wl.Window(1500, 300, 1)
    nu_first, dnu = oracle.window_grid(tab, w)
    edges = wl.snapped_edges(tab, w, wl.log_edges(nu_first + 40 * dnu, nu_first + 260 * dnu, 4))
    obs = hr2.Obs(ctx, T, w, 400.0, edges)
    col = tu.small_columns(tab, 1, seed=1024, n_levels=1024)[0]
    ref = oracle.forward(tab, col, w, 400.0, edges, 3)
    for chunks in (1, 0, 8):
        say(f"1024 levels {dtype} chunks={chunks}")
        bins, fplus = run_forward(ctx, T, obs, [col], 3, chunks)
        e_f, _ = tu.max_rel_err(fplus[0], ref["fplus"])
        e_b, _ = tu.max_rel_err(bins[0], ref["bins"])
        assert e_f <= tol and e_b <= tol, (dtype, chunks, e_f, e_b)
    obs.close()
    T.close()


@pytest.mark.parametrize("dtype,tol", [("f64", 1e-12), ("f32", 1e-5)])
def test_zigzag_temperature_profiles(ctx, dtype, tol):
    """Temperature profiles that cross the table's T nodes back and forth
    (and leave the axis at both ends), so that table rows leave the cell and
    come back in both sweep directions: the row masks for upward and
    downward layer chunks must fetch exactly what the slots lack."""
    tab = tu.small_multi_table()
    T = hr2.Tables(ctx, tab, dtype)
    w = wl.Window(3, 2990, 1)
    nu_first, dnu = oracle.window_grid(tab, w)
    edges = wl.snapped_edges(tab, w, wl.log_edges(nu_first + 200 * dnu, nu_first + 2700 * dnu, 7))
    obs = hr2.Obs(ctx, T, w, 400.0, edges)
    rng = np.random.default_rng(11)
    cols = []
    for L, period, amp in ((57, 5.0, 1300.0), (33, 2.3, 900.0), (64, 9.7, 1600.0)):
        p = wl.levels(L, 2.3, -4.7)
        lev = np.arange(L)
        Tk = np.clip(1500.0 + amp * np.sin(2 * np.pi * lev / period + rng.uniform(0, 6)), 120.0, 3400.0)
        x = wl.log_uniform(rng, 1e-6, 1e-2, tab.n_species)
        cols.append(wl.Column(p, Tk, x, 4.5, wl.scale_factor(1.0)))
    refs = [oracle.forward(tab, c, w, 400.0, edges, 3) for c in cols]
    for chunks in (1, 2, 3, 4, 5, 8):
        for s, col in enumerate(cols):
            say(f"zigzag {dtype} L={col.n_levels} chunks={chunks}")
            bins, fplus = run_forward(ctx, T, obs, [col], 3, chunks)
            e_f, _ = tu.max_rel_err(fplus[0], refs[s]["fplus"])
            e_b, _ = tu.max_rel_err(bins[0], refs[s]["bins"])
            assert e_f <= tol and e_b <= tol, (dtype, chunks, s, e_f, e_b)
    obs.close()
    T.close()


def test_isothermal_and_transparent_limits(ctx):
    """P3/P5 on the GPU: isothermal columns give pi B(T) at every point (FP32)."""
    tab = tu.c1_table()
    T = hr2.Tables(ctx, tab, "f32")
    p = wl.levels(21, 2.0, -4.0)
    w = wl.Window(0, tab.n_nu, 1)
    spec = wl.c1_obs(tab)
    obs = hr2.Obs(ctx, T, w, 300.0, spec.edges_cm)
    cols = [wl.Column(p, np.full(21, t), np.array([1e-3]), 4.75, 1.0) for t in (300.0, 900.0, 1733.0)]
    say("isothermal columns, f32")
    _, fplus = run_forward(ctx, T, obs, cols)
    nu = tab.nu(0, tab.n_nu, 1)
    for s, c in enumerate(cols):
        ref = np.pi * oracle.planck(nu, np.full(nu.shape, c.T_K[0]))
        e, _ = tu.max_rel_err(fplus[s], ref)
        say(f"  T={c.T_K[0]}: {e:.2e}")
        assert e <= 1e-5


@pytest.mark.parametrize("dtype,tol", [("f64", 1e-12), ("f32", 1e-5)])
def test_cold_upper_levels(ctx, dtype, tol):
    """Levels far below the table's T axis (down to 25 K): c2 nu / T reaches
    ~350 at 6000 cm^-1, beyond the FP32 exponent range, and the Planck
    function of those levels must come out 0-ish, never inf or NaN."""
    tab = tu.c1_table()
    spec = wl.c1_obs(tab)
    p = wl.levels(21, 2.0, -4.0)
    cols = [wl.Column(p, wl.linear_logp_profile(p, Tb, Tt), np.array([1e-3]), 4.75,
                      wl.scale_factor(1.0)) for Tb, Tt in ((1400.0, 25.0), (900.0, 60.0))]
    T = hr2.Tables(ctx, tab, dtype)
    obs = hr2.Obs(ctx, T, spec.window, spec.resolving_power, spec.edges_cm)
    bins, fplus = run_forward(ctx, T, obs, cols)
    assert np.all(np.isfinite(bins)) and np.all(np.isfinite(fplus))
    for s, col in enumerate(cols):
        ref = oracle.forward(tab, col, spec.window, spec.resolving_power, spec.edges_cm, 3)
        e_f, _ = tu.max_rel_err(fplus[s], ref["fplus"])
        e_b, _ = tu.max_rel_err(bins[s], ref["bins"])
        say(f"  cold set {s} {dtype}: F+ {e_f:.2e} bins {e_b:.2e}")
        assert e_f <= tol and e_b <= tol
    obs.close()
    T.close()


def test_batch_independence_and_device_entry(ctx):
    """P15: a set's result does not depend on the other sets of the launch
    (bit-identical), and the device-column entry equals the host entry."""
    tab = tu.c1_table()
    T = hr2.Tables(ctx, tab, "f32")
    spec = wl.c1_obs(tab)
    obs = hr2.Obs(ctx, T, spec.window, spec.resolving_power, spec.edges_cm)
    cols = wl.c3_columns(64, seed=9)
    say("batch of 64 vs singles (chunks fixed at 1)")
    bins_b, fp_b = run_forward(ctx, T, obs, cols, 3, chunks=1)
    for s in (0, 17, 63):
        b1, f1 = run_forward(ctx, T, obs, [cols[s]], 3, chunks=1)
        assert np.array_equal(b1[0], bins_b[s]) and np.array_equal(f1[0], fp_b[s])
    say("device-column entry")
    B, L = len(cols), cols[0].n_levels
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()
    p = dev(np.stack([c.p_bar for c in cols]))
    Tk = dev(np.stack([c.T_K for c in cols]))
    x = dev(np.stack([c.x for c in cols]))
    lg = dev([c.log_g for c in cols])
    sc = dev([c.scale for c in cols])
    bins = torch.empty(B * obs.n_bins, dtype=torch.float32, device="cuda")
    status = torch.full((B,), 7, dtype=torch.int32, device="cuda")
    ctx.set_option(hr2.OPT_CHUNKS, 1)
    hr2.forward_batch_dev(ctx, T, obs, p, Tk, x, lg, sc, 3, bins, None, status)
    torch.cuda.synchronize()
    assert np.array_equal(bins.cpu().numpy().reshape(B, -1), bins_b.astype(np.float32))
    assert int(status.abs().sum()) == 0
    say("device-column entry with one invalid set")
    Tbad = Tk.clone()
    Tbad[5, 3] = -10.0
    hr2.forward_batch_dev(ctx, T, obs, p, Tbad, x, lg, sc, 3, bins, None, status)
    torch.cuda.synchronize()
    out = bins.cpu().numpy().reshape(B, -1)
    st = status.cpu().numpy()
    assert st[5] == hr2.E_INVALID_ARG and np.all(np.delete(st, 5) == 0)
    assert np.all(np.isnan(out[5]))
    assert np.array_equal(np.delete(out, 5, axis=0), np.delete(bins_b.astype(np.float32), 5, axis=0))
    ctx.set_option(hr2.OPT_CHUNKS, 0)


def test_c3_batch_512(ctx):
    """C3: 512 sets on the C1 grid in one launch; every 31st set against the oracle."""
    tab = tu.c1_table()
    T = hr2.Tables(ctx, tab, "f32")
    spec = wl.c1_obs(tab)
    obs = hr2.Obs(ctx, T, spec.window, spec.resolving_power, spec.edges_cm)
    cols = wl.c3_columns()
    say("C3 512 sets f32")
    bins, fplus = run_forward(ctx, T, obs, cols)
    worst = 0.0
    for s in range(0, 512, 31):
        ref = oracle.forward(tab, cols[s], spec.window, spec.resolving_power, spec.edges_cm, 3)
        e_b, _ = tu.max_rel_err(bins[s], ref["bins"])
        e_f, _ = tu.max_rel_err(fplus[s], ref["fplus"])
        worst = max(worst, e_b, e_f)
    say(f"  worst {worst:.2e}")
    assert worst <= 1e-5


def test_abi_errors_leave_outputs_untouched(ctx):
    """Invalid arguments return the documented codes before anything is enqueued."""
    tab = tu.c1_table()
    T = hr2.Tables(ctx, tab, "f32")
    spec = wl.c1_obs(tab)
    obs = hr2.Obs(ctx, T, spec.window, spec.resolving_power, spec.edges_cm)
    good = wl.c1_columns()[2]
    bins = torch.full((obs.n_bins,), 123.0, dtype=torch.float32, device="cuda")

    def expect(status, cols, n_mu=3):
        with pytest.raises(hr2.HR2Error) as ei:
            hr2.forward_batch(ctx, T, obs, cols, n_mu, bins)
        assert ei.value.status == status, ei.value

    bad_T = wl.Column(good.p_bar, good.T_K.copy(), good.x, good.log_g, good.scale)
    bad_T.T_K[4] = np.nan
    expect(hr2.E_INVALID_ARG, [bad_T])
    bad_p = wl.Column(good.p_bar[::-1].copy(), good.T_K, good.x, good.log_g, good.scale)
    expect(hr2.E_INVALID_ARG, [bad_p])
    expect(hr2.E_INVALID_ARG, [wl.Column(good.p_bar, good.T_K, np.array([1.5]), 4.0, 1.0)])
    expect(hr2.E_OUT_OF_RANGE, [good], n_mu=0)
    expect(hr2.E_OUT_OF_RANGE, [good], n_mu=9)
    short = wl.Column(good.p_bar[:1], good.T_K[:1], good.x, good.log_g, good.scale)
    expect(hr2.E_INVALID_ARG, [short])
    torch.cuda.synchronize()
    assert torch.all(bins == 123.0)
    with pytest.raises(hr2.HR2Error) as ei:
        hr2.Obs(ctx, T, wl.Window(0, 3000, 1), 300.0, spec.edges_cm)
    assert ei.value.status == hr2.E_OUT_OF_RANGE
    with pytest.raises(hr2.HR2Error) as ei:
        hr2.Obs(ctx, T, spec.window, 300.0, [4100.0, 4100.2, 4300.0])
    assert ei.value.status == hr2.E_INVALID_ARG


@pytest.mark.parametrize("dtype,tol", [("f64", 1e-12), ("f32", 1e-5)])
def test_degenerate_sizes(ctx, dtype, tol):
    """An empty batch and an empty window are refused before anything runs;
    the smallest windows (two and three points in one bin), one-layer and
    two-layer columns, one angle, and one full tile plus a one-point tail
    match the oracle through every chunking."""
    tab = tu.small_multi_table()
    T = hr2.Tables(ctx, tab, dtype)
    w0 = wl.Window(10, 200, 1)
    nu0, d0 = oracle.window_grid(tab, w0)
    obs0 = hr2.Obs(ctx, T, w0, 300.0, [nu0 + 20 * d0, nu0 + 150 * d0])
    bins0 = torch.full((obs0.n_bins,), 7.0, dtype=T.real, device="cuda")
    with pytest.raises(hr2.HR2Error) as ei:
        hr2.forward_batch(ctx, T, obs0, [], 3, bins0)
    assert ei.value.status == hr2.E_INVALID_ARG
    torch.cuda.synchronize()
    assert torch.all(bins0 == 7.0)
    obs0.close()
    with pytest.raises(hr2.HR2Error) as ei:
        hr2.Obs(ctx, T, wl.Window(10, 0, 1), 300.0, [nu0, nu0 + d0])
    assert ei.value.status == hr2.E_OUT_OF_RANGE
    cases = [(wl.Window(500, 2, 1), 2, 1), (wl.Window(77, 3, 5), 2, 3),
             (wl.Window(5, 65, 3), 3, 1), (wl.Window(1000, 65, 1), 41, 8)]
    for w, L, n_mu in cases:
        cols = tu.small_columns(tab, 2, seed=L + w.count, n_levels=L)
        nu_first, dnu = oracle.window_grid(tab, w)
        edges = [nu_first, nu_first + (w.count - 1) * dnu]
        obs = hr2.Obs(ctx, T, w, 300.0, edges)
        refs = [oracle.forward(tab, c, w, 300.0, edges, n_mu) for c in cols]
        for chunks in (0, 1, 3):
            bins, fplus = run_forward(ctx, T, obs, cols, n_mu, chunks)
            for s, ref in enumerate(refs):
                e_f, _ = tu.max_rel_err(fplus[s], ref["fplus"])
                e_b, _ = tu.max_rel_err(bins[s], ref["bins"])
                assert e_f <= tol and e_b <= tol, (w, L, n_mu, chunks, s, e_f, e_b)
        say(f"{dtype} window {w} L={L} n_mu={n_mu}: ok")
        obs.close()
    ctx.set_option(hr2.OPT_CHUNKS, 0)
    T.close()


def test_row_policy_leaves_results_unchanged(ctx):
    """HR2_OPT_ROW_POLICY only changes how one-set calls load table rows:
    non-temporal and cached loads give bit-identical spectra and bins."""
    tab = tu.small_multi_table()
    T = hr2.Tables(ctx, tab, "f32")
    w = wl.Window(13, 1001, 2)
    nu_first, dnu = oracle.window_grid(tab, w)
    obs = hr2.Obs(ctx, T, w, 400.0, wl.snapped_edges(
        tab, w, wl.log_edges(nu_first + 0.2 * (w.count - 1) * dnu,
                             nu_first + 0.8 * (w.count - 1) * dnu, 9)))
    col = tu.small_columns(tab, 1, seed=31)
    out = {}
    for policy in (1, 2, 0):
        ctx.set_option(hr2.OPT_ROW_POLICY, policy)
        out[policy] = run_forward(ctx, T, obs, col, 3, 2)
    ctx.set_option(hr2.OPT_CHUNKS, 0)
    for policy in (2, 0):
        assert np.array_equal(out[1][0], out[policy][0])
        assert np.array_equal(out[1][1], out[policy][1])
    with pytest.raises(hr2.HR2Error) as ei:
        ctx.set_option(hr2.OPT_ROW_POLICY, 3)
    assert ei.value.status == hr2.E_INVALID_ARG
    obs.close()
    T.close()


# C2 / C4 at full size: tests/test_gpu_fullsize.py


def test_c3_graph_replay(ctx):
    """C3 as a HIP graph: the 512-set batch captured once and replayed, with
    eager work and synchronisations between replays, equals the eager launch."""
    tab = tu.c1_table()
    T = hr2.Tables(ctx, tab, "f32")
    spec = wl.c1_obs(tab)
    obs = hr2.Obs(ctx, T, spec.window, spec.resolving_power, spec.edges_cm)
    cols = wl.c3_columns()
    B = len(cols)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()
    p = dev(np.stack([c.p_bar for c in cols]))
    Tk = dev(np.stack([c.T_K for c in cols]))
    x = dev(np.stack([c.x for c in cols]))
    lg = dev([c.log_g for c in cols])
    sc = dev([c.scale for c in cols])
    bins = torch.empty(B * obs.n_bins, dtype=torch.float32, device="cuda")
    fplus = torch.empty(B * spec.window.count, dtype=torch.float32, device="cuda")
    ctx.set_option(hr2.OPT_CHUNKS, 0)
    say("C3 eager")
    hr2.forward_batch_dev(ctx, T, obs, p, Tk, x, lg, sc, 3, bins, fplus)
    torch.cuda.synchronize()
    ref = bins.clone()
    say("C3 capture")
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            hr2.forward_batch_dev(ctx, T, obs, p, Tk, x, lg, sc, 3, bins, fplus, None, s)
    torch.cuda.synchronize()
    for rep in range(3):
        bins.zero_()
        junk = torch.randn(1 << 16, device="cuda").sum()
        torch.cuda.synchronize()
        say(f"C3 replay {rep}")
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(bins, ref), rep
        del junk
    del g
    torch.cuda.synchronize()


@pytest.mark.parametrize("dtype", ["f32", "f16", "bf16"])
def test_whole_forward_per_set(ctx, dtype):
    """Small windows in batches that fill the device (one-species tables) run
    the whole forward model in one launch, one workgroup per set (levels and
    F+ in LDS), with one or two wavenumbers per lane.  Both must agree with the
    three-kernel path (forced by a fixed chunk count) to FP32 rounding (5e-6)
    and with the oracle at every tested set (1e-5), for both angle tiers, with a ragged
    last tile and with an invalid set in the batch."""
    tab = tu.c1_table()
    T = hr2.Tables(ctx, tab, dtype)
    ref_tab = tab if dtype == "f32" else tu.dequantised(tab, dtype)
    w = wl.Window(3, 1990, 1)   # 15.5 tiles of 128 points, 31.1 of 64
    nu_first, dnu = oracle.window_grid(tab, w)
    edges = wl.snapped_edges(tab, w, wl.log_edges(nu_first + 100 * dnu, nu_first + 1880 * dnu, 30))
    obs = hr2.Obs(ctx, T, w, 2000.0, edges)
    B = 300   # 300 sets x 32 tiles: more waves than the device holds at once
    cols = tu.small_columns(tab, B, seed=77, n_levels=41)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()
    p = dev(np.stack([c.p_bar for c in cols]))
    Tk = dev(np.stack([c.T_K for c in cols]))
    x = dev(np.stack([c.x for c in cols]))
    lg = dev([c.log_g for c in cols])
    sc = dev([c.scale for c in cols])
    bins = torch.empty(B * obs.n_bins, dtype=torch.float32, device="cuda")
    fplus = torch.empty(B * w.count, dtype=torch.float32, device="cuda")
    status = torch.full((B,), 7, dtype=torch.int32, device="cuda")

    def run(n_mu, chunks, per_lane):
        ctx.set_option(hr2.OPT_CHUNKS, chunks)
        ctx.set_option(hr2.OPT_NU_PER_LANE, per_lane)
        hr2.forward_batch_dev(ctx, T, obs, p, Tk, x, lg, sc, n_mu, bins, fplus, status)
        torch.cuda.synchronize()
        ctx.set_option(hr2.OPT_CHUNKS, 0)
        ctx.set_option(hr2.OPT_NU_PER_LANE, 0)
        assert int(status.abs().sum()) == 0
        return (bins.cpu().numpy().reshape(B, -1).astype(np.float64),
                fplus.cpu().numpy().reshape(B, -1).astype(np.float64))

    for n_mu in (3, 5):
        three = run(n_mu, 1, 0)
        for per_lane in (1, 2):
            got = run(n_mu, 0, per_lane)
            d_b = np.max(np.abs(got[0] - three[0]) / np.abs(three[0]))
            d_f = np.max(np.abs(got[1] - three[1]) / np.abs(three[1]))
            say(f"per-set launch {dtype} n_mu={n_mu}, {per_lane} per lane: vs three kernels "
                f"bins {d_b:.1e}, F+ {d_f:.1e}")
            # two FP32 evaluations of one recurrence, each ~1e-6 from the
            # oracle's FP64 value: at most about twice that apart
            assert d_b <= 5e-6 and d_f <= 5e-6
            for s in (0, 150, B - 1):
                ref = oracle.forward(ref_tab, cols[s], w, 2000.0, edges, n_mu)
                e_f, _ = tu.max_rel_err(got[1][s], ref["fplus"])
                e_b, _ = tu.max_rel_err(got[0][s], ref["bins"])
                say(f"  set {s}: F+ {e_f:.2e} bins {e_b:.2e}")
                assert e_f <= 1e-5 and e_b <= 1e-5
    say("one invalid set in the batch")
    valid = run(5, 0, 0)
    Tbad = Tk.clone()
    Tbad[7, 3] = -10.0
    hr2.forward_batch_dev(ctx, T, obs, p, Tbad, x, lg, sc, 5, bins, fplus, status)
    torch.cuda.synchronize()
    got = bins.cpu().numpy().reshape(B, -1).astype(np.float64)
    st = status.cpu().numpy()
    assert st[7] == hr2.E_INVALID_ARG and np.all(np.delete(st, 7) == 0)
    assert np.all(np.isnan(got[7]))
    assert np.array_equal(np.delete(got, 7, axis=0), np.delete(valid[0], 7, axis=0))
    with pytest.raises(hr2.HR2Error) as ei:
        ctx.set_option(hr2.OPT_NU_PER_LANE, 3)
    assert ei.value.status == hr2.E_UNSUPPORTED
    obs.close()
    T.close()


def test_kernel_timing_leaves_results_unchanged(ctx):
    """HR2_OPT_TIMING times every n-th call's kernels through HIP events
    attached to their launches: the call count, three positive intervals, the
    column kernel alone with HR2_OPT_TIMING_KERNELS = 2, bad masks refused,
    and results bit-identical to untimed calls."""
    tab = tu.c1_table()
    T = hr2.Tables(ctx, tab, "f32")
    spec = wl.c1_obs(tab)
    obs = hr2.Obs(ctx, T, spec.window, spec.resolving_power, spec.edges_cm)
    col = wl.c1_columns()[:1]
    ref = run_forward(ctx, T, obs, col, 3)
    ctx.set_option(hr2.OPT_TIMING, 2)
    ctx.collect_timing()
    outs = [run_forward(ctx, T, obs, col, 3) for _ in range(5)]
    ctx.set_option(hr2.OPT_TIMING, 0)
    (ms_lev, ms_col, ms_conv), n = ctx.collect_timing()
    say(f"  timed calls {n}: levels {ms_lev / n * 1e3:.1f} us, column {ms_col / n * 1e3:.1f} us, "
        f"convolution {ms_conv / n * 1e3:.1f} us per call")
    assert n == 3
    assert ms_lev > 0 and ms_col > 0 and ms_conv > 0
    for b, f in outs:
        assert np.array_equal(b, ref[0]) and np.array_equal(f, ref[1])
    (z0, z1, z2), n0 = ctx.collect_timing()
    assert n0 == 0 and z0 == z1 == z2 == 0.0
    # the column kernel alone (HR2_OPT_TIMING_KERNELS = 2), then a bad mask
    ctx.set_option(hr2.OPT_TIMING, 1)
    ctx.set_option(hr2.OPT_TIMING_KERNELS, 2)
    outs = [run_forward(ctx, T, obs, col, 3) for _ in range(2)]
    ctx.set_option(hr2.OPT_TIMING, 0)
    (c0, c1, c2), n = ctx.collect_timing()
    assert n == 2 and c0 == 0.0 and c1 > 0 and c2 == 0.0
    for b, f in outs:
        assert np.array_equal(b, ref[0]) and np.array_equal(f, ref[1])
    for bad in (0, 8):
        with pytest.raises(hr2.HR2Error) as ei:
            ctx.set_option(hr2.OPT_TIMING_KERNELS, bad)
        assert ei.value.status == hr2.E_INVALID_ARG
    ctx.set_option(hr2.OPT_TIMING_KERNELS, 7)
    obs.close()
    T.close()
