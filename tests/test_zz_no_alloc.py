"""The allocation-free entry point (hr2_forward_batch_dev_noalloc) against
hr2_forward_batch_dev: the same kernels on the same inputs, so bins and F+
must agree bit for bit; two calls in a row, the second smaller, and a call
too large for the fixed array refused before anything runs."""
import numpy as np
import pytest

import workloads as wl
from tests import hr2_testutil as tu

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_1910_01070_amd import hr2  # noqa: E402


def say(*a):
    print(*a, flush=True)


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def _columns(cols):
    return (_dev(np.stack([c.p_bar for c in cols])), _dev(np.stack([c.T_K for c in cols])),
            _dev(np.stack([c.x for c in cols])), _dev([c.log_g for c in cols]),
            _dev([c.scale for c in cols]))


def _both(ctx, T, obs, cols, n_mu):
    """bins and F+ of the existing entry point, then of the allocation-free one
    (F+ once in the fixed array, once in a caller buffer)."""
    B = len(cols)
    p, Tk, x, lg, sc = _columns(cols)
    nb, nf = B * obs.n_bins, B * obs.window.count
    ref_b = torch.empty(nb, dtype=T.real, device="cuda")
    ref_f = torch.empty(nf, dtype=T.real, device="cuda")
    hr2.forward_batch_dev(ctx, T, obs, p, Tk, x, lg, sc, n_mu, ref_b, ref_f)
    got_b = torch.full((nb,), -1.0, dtype=T.real, device="cuda")
    status = torch.full((B,), 7, dtype=torch.int32, device="cuda")
    hr2.forward_batch_dev_noalloc(ctx, T, obs, p, Tk, x, lg, sc, n_mu, got_b, None, status)
    got_b2 = torch.full((nb,), -1.0, dtype=T.real, device="cuda")
    got_f = torch.full((nf,), -1.0, dtype=T.real, device="cuda")
    hr2.forward_batch_dev_noalloc(ctx, T, obs, p, Tk, x, lg, sc, n_mu, got_b2, got_f)
    torch.cuda.synchronize()
    assert int(status.abs().sum()) == 0
    return ref_b.cpu(), ref_f.cpu(), got_b.cpu(), got_b2.cpu(), got_f.cpu()


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_noalloc_matches_forward_batch_dev(dtype):
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    ctx = hr2.Context(0)
    tab = tu.small_multi_table()
    T = hr2.Tables(ctx, tab, dtype)
    cases = [(wl.Window(0, 3000, 1), 41, 6, 3), (wl.Window(13, 1001, 2), 23, 2, 5)]
    for w, L, B, n_mu in cases:
        nu_first = tab.nu0_cm + w.begin * tab.dnu_cm
        dnu = w.stride * tab.dnu_cm
        edges = wl.snapped_edges(tab, w, wl.log_edges(nu_first + 0.2 * (w.count - 1) * dnu,
                                                     nu_first + 0.8 * (w.count - 1) * dnu, 9))
        obs = hr2.Obs(ctx, T, w, 400.0, edges)
        cols = tu.small_columns(tab, B, seed=L + B, n_levels=L)
        say(f"noalloc {dtype}: window {w}, {L} levels, {B} sets, {n_mu} angles")
        ref_b, ref_f, got_b, got_b2, got_f = _both(ctx, T, obs, cols, n_mu)
        assert torch.isfinite(ref_b).all()
        assert torch.equal(got_b, ref_b), (w, L, B)
        assert torch.equal(got_b2, ref_b), (w, L, B)
        assert torch.equal(got_f, ref_f), (w, L, B)
        obs.close()
    T.close()
    ctx.close()


def test_noalloc_refuses_a_call_beyond_its_array():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    ctx = hr2.Context(0)
    tab = tu.small_multi_table()
    T = hr2.Tables(ctx, tab, "f32")
    w = wl.Window(0, 3000, 1)
    nu_first = tab.nu0_cm
    edges = wl.snapped_edges(tab, w, wl.log_edges(nu_first + 300 * tab.dnu_cm,
                                                 nu_first + 2700 * tab.dnu_cm, 5))
    obs = hr2.Obs(ctx, T, w, 400.0, edges)
    # 3000 sets of 41 levels: 15.7 MB of records + 36 MB of F+ > 32 MiB
    B, L = 3000, 41
    col = tu.small_columns(tab, 1, seed=3, n_levels=L)[0]
    p, Tk, x, lg, sc = _columns([col] * B)
    bins = torch.full((B * obs.n_bins,), 5.0, dtype=torch.float32, device="cuda")
    with pytest.raises(hr2.HR2Error) as ei:
        hr2.forward_batch_dev_noalloc(ctx, T, obs, p, Tk, x, lg, sc, 3, bins)
    assert ei.value.status == hr2.E_OUT_OF_RANGE
    assert "fixed array" in str(ei.value)
    torch.cuda.synchronize()
    assert torch.all(bins == 5.0)
    # with the caller's F+ buffer the records alone fit; the same call through
    # the regular entry point (same batch, so the same launch shape) agrees
    # bit for bit
    fplus = torch.empty(B * w.count, dtype=torch.float32, device="cuda")
    hr2.forward_batch_dev_noalloc(ctx, T, obs, p, Tk, x, lg, sc, 3, bins, fplus)
    ref = torch.empty_like(bins)
    ref_f = torch.empty_like(fplus)
    hr2.forward_batch_dev(ctx, T, obs, p, Tk, x, lg, sc, 3, ref, ref_f)
    torch.cuda.synchronize()
    assert torch.equal(bins.cpu(), ref.cpu()) and torch.equal(fplus.cpu(), ref_f.cpu())
    obs.close()
    T.close()
    ctx.close()


def test_noalloc_captured_into_a_graph_without_a_prior_call():
    """The entry point needs no staging and no scratch growth, so it can be
    captured into a HIP graph on a fresh context; every replay (with eager
    work and synchronisations between them) equals the eager call."""
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    ctx = hr2.Context(0)
    tab = tu.small_multi_table()
    T = hr2.Tables(ctx, tab, "f32")
    w = wl.Window(13, 1001, 2)
    nu_first = tab.nu0_cm + w.begin * tab.dnu_cm
    dnu = w.stride * tab.dnu_cm
    edges = wl.snapped_edges(tab, w, wl.log_edges(nu_first + 0.2 * (w.count - 1) * dnu,
                                                 nu_first + 0.8 * (w.count - 1) * dnu, 9))
    obs = hr2.Obs(ctx, T, w, 400.0, edges)
    cols = tu.small_columns(tab, 4, seed=41, n_levels=41)
    p, Tk, x, lg, sc = _columns(cols)
    bins = torch.empty(4 * obs.n_bins, dtype=torch.float32, device="cuda")
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            hr2.forward_batch_dev_noalloc(ctx, T, obs, p, Tk, x, lg, sc, 3, bins, None, None, s)
    torch.cuda.synchronize()
    ref = torch.empty_like(bins)
    hr2.forward_batch_dev(ctx, T, obs, p, Tk, x, lg, sc, 3, ref)
    torch.cuda.synchronize()
    for rep in range(3):
        bins.zero_()
        junk = torch.randn(1 << 16, device="cuda").sum()
        torch.cuda.synchronize()
        say(f"noalloc graph replay {rep}")
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(bins, ref), rep
        del junk
    del g
    torch.cuda.synchronize()
    obs.close()
    T.close()
    ctx.close()
