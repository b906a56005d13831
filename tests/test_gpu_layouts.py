"""GPU parity of the observation layout build (the 5 sigma half widths, the
normalisations Z_i and the banded per-bin weights of hr2_obs_create) through
hr2_convolve_bin, fed a fixed seeded spectrum.  Windows whose profile width
s = sigma / dnu crosses 4 grid steps (where FP32 layouts switch from direct
sums to the closed form), strided windows (s < 4 throughout), very wide
profiles (s in the tens to a hundred), bins reaching the window's ends, and a
single bin over the whole window.  Oracle: direct convolution, then binning
(FP64).  Tolerances: 1e-12 (FP64 layouts), 1e-5 (FP32)."""
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


def profile_widths(tab, w, R):
    nu_first, dnu = oracle.window_grid(tab, w)
    nu_last = nu_first + (w.count - 1) * dnu
    c = 1.0 / (R * 2.0 * np.sqrt(2.0 * np.log(2.0)) * dnu)
    return nu_first * c, nu_last * c


@pytest.mark.parametrize("dtype,tol", [("f64", 1e-12), ("f32", 1e-5)])
def test_layouts_across_profile_widths(ctx, dtype, tol):
    tab = tu.small_multi_table()
    T = hr2.Tables(ctx, tab, dtype)
    cases = [
        (wl.Window(0, 3000, 1), 480.0, "inner", 9),    # s 3.5 .. 6.2: crosses 4
        (wl.Window(0, 3000, 1), 30.0, "ends", 7),      # s 57 .. 99, bins to the ends
        (wl.Window(3, 400, 7), 150.0, "inner", 5),     # strided, s 1.6 .. 2.8
        (wl.Window(40, 1400, 2), 90.0, "ends", 1),     # one bin over the window
    ]
    rng = np.random.default_rng(77)
    for w, R, where, n_edges in cases:
        s_lo, s_hi = profile_widths(tab, w, R)
        nu_first, dnu = oracle.window_grid(tab, w)
        nu_last = nu_first + (w.count - 1) * dnu
        if where == "inner":
            lo, hi = nu_first + 0.2 * (nu_last - nu_first), nu_first + 0.8 * (nu_last - nu_first)
        else:
            lo, hi = nu_first + dnu, nu_last - dnu
        edges = wl.snapped_edges(tab, w, wl.log_edges(lo, hi, n_edges) if n_edges > 1
                                 else [lo, hi])
        obs = hr2.Obs(ctx, T, w, R, edges)
        F = 1.0 + 0.3 * np.sin(0.05 * np.arange(w.count)) + 0.2 * rng.random(w.count)
        fin = torch.from_numpy(F.astype(np.float64 if dtype == "f64" else np.float32)).cuda()
        bins = torch.empty(obs.n_bins, dtype=T.real, device="cuda")
        hr2.convolve_bin(ctx, obs, fin, 2.5, bins)
        torch.cuda.synchronize()
        idx = oracle.snap_edges(edges, nu_first, dnu, w.count)
        fd = np.zeros(w.count)
        # the same rounded input the device read
        Fr = fin.cpu().numpy().astype(np.float64)
        fd[idx[0]:idx[-1] + 1] = oracle.convolve(Fr, nu_first, dnu, R,
                                                 np.arange(idx[0], idx[-1] + 1))
        ref = oracle.bin_spectrum(fd, idx, nu_first, dnu, 2.5)
        e, _ = tu.max_rel_err(bins.cpu().numpy().astype(np.float64), ref)
        say(f"{dtype} window {w} R={R:g} s {s_lo:.1f}..{s_hi:.1f} bins {obs.n_bins}: {e:.2e}")
        assert e <= tol, (w, R, e)
        obs.close()
    T.close()
