"""Benchmark of the Helios-r2 emission forward model on one MI355X.

One step = one pass of the whole forward model over one batch of synthetic
columns already resident in HBM: level records, the fused opacity + RT
column kernel, the convolve/bin kernel (hr2_forward_batch_dev).

Default workload: a single realistic forward model at FP32 (8 absorbers +
H2-H2/H2-He CIA, 27 T x 19 log p table, 150,000 wavenumbers at 0.1 cm^-1,
100 layers, 3 angles, R = 300, 400 bins).  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "forward spectra/s and layer·ν points/s + p50/p99 latency vs plain FP32 at ≤1e-3"
HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def axis_cell(axis, v):
    """Table cell of the forward model's lookup rule (lower node = largest
    index with axis[i] <= v, clamped, capped at n-2) and the upper weight."""
    v = np.clip(v, axis[0], axis[-1])
    i = np.searchsorted(axis, v, side="right") - 1
    i = np.minimum(i, len(axis) - 2)
    w = (v - axis[i]) / (axis[i + 1] - axis[i])
    return i, w


def algorithmic_bytes(tab, cols, elem_bytes, n_nu, n_bins):
    """Bytes the column kernel must move: every distinct table row (T node,
    p node) with nonzero weight in any level of any set, per species, at
    elem_bytes per entry, plus the distinct CIA rows (FP32) and the F+ write."""
    rows, cia_rows = set(), set()
    for c in cols:
        iT, wT = axis_cell(tab.T_K, c.T_K)
        ip, wp = axis_cell(tab.log10_p_bar, np.log10(c.p_bar))
        for a in (0, 1):
            for b in (0, 1):
                w = (wT if a else 1 - wT) * (wp if b else 1 - wp)
                for k in np.nonzero(w)[0]:
                    rows.add((int(iT[k] + a), int(ip[k] + b)))
            wt = wT if a else 1 - wT
            for k in np.nonzero(wt)[0]:
                cia_rows.add(int(iT[k] + a))
    S = tab.n_species
    table = S * len(rows) * n_nu * elem_bytes
    cia = tab.n_cia * len(cia_rows) * n_nu * 4
    out = len(cols) * n_nu * 4
    return table + cia + out, len(rows), len(cia_rows)


def kernel_source_hash():
    h = hashlib.sha256()
    with open(os.path.join(ROOT, "paper_1910_01070_amd", "csrc", "kernels.hip"), "rb") as f:
        h.update(f.read())
    return h.hexdigest()[:16]


def traffic_from_profile(kernel_hash):
    """HBM bytes per launch of the column kernel from committed rocprofv3
    counter runs, if they were taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", "column_kernel_c2_f32_counters.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    if d.get("kernel_source_sha256_16") != kernel_hash:
        return None
    return d.get("hbm_bytes_per_launch")


def valu_from_profile(kernel_hash, col_ms):
    """The column kernel's VALU issue time per launch from a committed
    rocprofv3 SQ counter run on the current kernel source: wave instructions
    x 4 cycles (64 lanes on a 16-wide SIMD), transcendental ones (exp2, rcp)
    x 8 (half rate, measured by a microbenchmark on an MI355X), over the
    chip's 1024 SIMDs at 2.4 GHz, next to the measured kernel time."""
    path = os.path.join(ROOT, "profiles", "column_kernel_c2_f32_valu.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    if d.get("kernel_source_sha256_16") != kernel_hash:
        return None
    valu, trans = d["sq_insts_valu_per_launch"], d.get("sq_insts_valu_trans_f32", 0.0)
    t_us = (valu + trans) * 4.0 / (1024 * 2.4e9) * 1e6
    return {"sq_insts_valu_per_launch": valu, "sq_insts_valu_trans_f32": trans,
            "cycles_per_wave_instruction": {"valu": 4, "transcendental": 8},
            "valu_issue_us": t_us, "kernel_us": col_ms * 1e3,
            "issue_frac": t_us / (col_ms * 1e3), "source": "profiles/column_kernel_c2_f32_valu.json"}


def cpu_baseline(tab, col, spec, n_mu, budget_s=20.0):
    """The FP64 oracle on the host cores: whole spectra of the same workload,
    repeated until about budget_s seconds have passed (at least one)."""
    import oracle
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    n = 0
    t0 = time.perf_counter()
    while True:
        oracle.forward(tab, col, spec.window, spec.resolving_power, spec.edges_cm, n_mu)
        n += 1
        el = time.perf_counter() - t0
        if el >= budget_s or el / n * (n + 1) > 1.5 * budget_s:
            break
    return {"value": n / el, "unit": "spectra/s", "cores": threads, "kind": "oracle",
            "sample": f"{n} whole spectra of the same workload (all stages, FP64), {el:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--dtype", default="f32", choices=["f32", "f16", "bf16"])
    ap.add_argument("--batch", type=int, default=1)
    ap.add_argument("--n-nu", type=int, default=150_000)
    ap.add_argument("--chunks", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget-s", type=float, default=20.0)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 1 GiB device-to-device copy 5 times (counter scale)")
    ap.add_argument("--workload", default="c2",
                    choices=["c1", "c2", "c3", "c4", "c5", "params", "oracle"],
                    help="c2 (default): one realistic spectrum per step; c1: one small FP64 "
                         "spectrum per synchronous call (latency); c3: 512-set C1 batch "
                         "as a HIP graph vs 512 sequential calls; c4: reduced-precision "
                         "batches; c5: Poisson serving trace; params: parameter vectors "
                         "to ln L; oracle: the FP64 oracle timed on the host")
    ap.add_argument("--source", type=int, default=1, choices=[1, 2],
                    help="short-characteristics source interpolant: 1 linear, 2 parabolic")
    ap.add_argument("--cloud", action="store_true",
                    help="c2: add a gray cloud (tau 5, top 0.3 bar, bottom 3 bar) to the column")
    ap.add_argument("--rate", type=float, default=2000.0, help="c5 arrival rate, requests/s")
    ap.add_argument("--duration", type=float, default=10.0, help="c5 trace length, s")
    ap.add_argument("--rates", default="", help="c5: comma-separated arrival rates to sweep")
    ap.add_argument("--strided-frac", type=float, default=0.5,
                    help="c5: share of requests on 1 cm^-1 windows (stride 10)")
    ap.add_argument("--no-comparison", action="store_true",
                    help="c2: skip the serving / plain FP32 / batch comparison legs")
    ap.add_argument("--cmp-rate", type=float, default=2000.0,
                    help="c2 comparison leg: arrival rate of the short serving trace")
    ap.add_argument("--cmp-duration", type=float, default=2.0,
                    help="c2 comparison leg: length of the short serving trace, s")
    ap.add_argument("--cmp-plain", type=int, default=200,
                    help="c2 comparison leg: requests timed on the plain FP32 path")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU; --gpus must be 1"}))
        sys.exit(2)
    if args.workload == "oracle":
        return run_oracle_timing(args)   # host only

    import torch
    import workloads as wl
    from paper_1910_01070_amd import hr2

    assert torch.cuda.is_available(), "bench needs a HIP device"
    if args.calibrate_copy:
        n = (1 << 30) // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"calibrate_copy_bytes_read": n * 4, "bytes_written": n * 4, "repeats": 5}))
        return
    if args.workload == "c1":
        return run_c1(args)
    if args.workload == "c3":
        return run_c3(args)
    if args.workload == "c4":
        return run_c4(args)
    if args.workload == "c5":
        return run_c5(args)
    if args.workload == "params":
        return run_params(args)
    log("generating tables")
    t0 = time.perf_counter()
    tab = wl.c2_table(n_nu=args.n_nu)
    log(f"  {time.perf_counter() - t0:.1f} s")
    spec = wl.c2_obs(tab)
    cols = [wl.c2_column()] if args.batch == 1 else wl.c4_columns(args.batch)
    if args.cloud:
        cols = [wl.Column(c.p_bar, c.T_K, c.x, c.log_g, c.scale, (5.0, 0.3, 10.0)) for c in cols]
    B, L = len(cols), cols[0].n_levels
    n_mu = 3

    ctx = hr2.Context(0)
    ctx.set_option(hr2.OPT_CHUNKS, args.chunks)
    ctx.set_option(hr2.OPT_SOURCE, args.source)
    T = hr2.Tables(ctx, tab, args.dtype)
    obs = hr2.Obs(ctx, T, spec.window, spec.resolving_power, spec.edges_cm)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()
    p = dev(np.stack([c.p_bar for c in cols]))
    Tk = dev(np.stack([c.T_K for c in cols]))
    x = dev(np.stack([c.x for c in cols]))
    lg = dev([c.log_g for c in cols])
    sc = dev([c.scale for c in cols])
    cl = dev([c.cloud for c in cols]) if args.cloud else None
    bins = torch.empty(B * obs.n_bins, dtype=torch.float32, device="cuda")
    fplus = torch.empty(B * spec.window.count, dtype=torch.float32, device="cuda")
    stream = torch.cuda.current_stream()

    def step():
        hr2.forward_batch_dev(ctx, T, obs, p, Tk, x, lg, sc, n_mu, bins, fplus, None, stream,
                              cloud=cl)

    default_launch = (args.source == 1 and not args.cloud and args.dtype == "f32" and B == 1
                      and args.n_nu == 150_000)
    default_c2 = default_launch and args.chunks == 0
    comparison, T16 = None, None
    if default_c2 and not args.no_comparison:
        # the comparison legs run first: besides their own figures, they leave
        # the device in the steady state of a loaded server (clocks up, the
        # FP32 table recently read by the batch leg) before the headline's
        # warmup and timed steps; from a cold start the column kernel needs
        # 100-200 steps to settle
        T16, comparison = comparison_legs(ctx, T, tab, args)

    # latency: one step at a time, host launch to device completion
    lat = []
    for k in range(min(args.steps, 200)):
        t1 = time.perf_counter()
        step()
        torch.cuda.synchronize()
        lat.append((time.perf_counter() - t1) * 1e3)
    lat = np.array(lat)
    # all three kernels of 16 more steps, each timed (outside every measurement)
    ctx.set_option(hr2.OPT_TIMING, 1)
    ctx.set_option(hr2.OPT_TIMING_KERNELS, 7)
    for k in range(16):
        step()
    ctx.set_option(hr2.OPT_TIMING, 0)
    (ms_lev, ms_col_b, ms_conv), n_break = ctx.collect_timing()

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    # timed region: K steps back to back; the library times the column
    # kernel of every 8th step from the second on (1, 9, 17, ...) through HIP
    # events attached to its launch on the launch stream.  One timed launch
    # costs ~5 us of GPU time, so the other two kernels are timed in the pass
    # of their own above; the first step, which follows the host's
    # synchronisation and runs a few us slower than the rest, stays out of
    # the three-launch sample (it counts in the wall-clock rate like any step).
    ctx.set_option(hr2.OPT_TIMING, 0)
    ctx.set_option(hr2.OPT_TIMING_KERNELS, 2)
    ctx.collect_timing()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        step()
        if k == 0:
            ctx.set_option(hr2.OPT_TIMING, 8)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ctx.set_option(hr2.OPT_TIMING, 0)
    (_, ms_col, _), n_timed = ctx.collect_timing()
    if T16 is not None:
        T16.close()   # freed only now: a free synchronises the device

    spectra_s = B * args.steps / wall
    layer_nu = (L - 1) * spec.window.count
    elem = {"f32": 4, "f16": 2, "bf16": 2}[args.dtype]
    alg_bytes, U, U_cia = algorithmic_bytes(tab, cols, elem, spec.window.count, obs.n_bins)
    col_ms = ms_col / max(n_timed, 1)
    achieved = alg_bytes / (col_ms * 1e-3) / 1e9
    khash = kernel_source_hash()
    traffic = traffic_from_profile(khash) if default_launch else None
    valu = valu_from_profile(khash, col_ms) if default_launch else None

    res = {
        "metric": METRIC,
        "value": spectra_s,
        "unit": "spectra/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.dtype == "f32" else f"f32 ({args.dtype} tables)",
        "data": "synthetic",
        "config": {
            "workload": ("single realistic forward model: 8 absorbers + H2-H2/H2-He CIA, "
                         "27 T x 19 log p table, 150k wavenumbers at 0.1 cm^-1, 100 layers, "
                         "6-knot T(p), 3 angles, R=300, 400 bins" if args.n_nu == 150_000 and B == 1
                         else f"C2-like batch of {B}, {args.n_nu} wavenumbers"),
            "sets_per_step": B, "layers": L - 1, "wavenumbers": spec.window.count,
            "species": tab.n_species, "cia_pairs": tab.n_cia, "n_mu": n_mu,
            "resolving_power": spec.resolving_power, "bins": obs.n_bins,
            "table_storage": args.dtype, "chunks": args.chunks,
            "source": "parabolic" if args.source == 2 else "linear",
            "cloud": "tau 5, 0.3-3 bar" if args.cloud else None,
        },
        "layer_nu_points_per_s": spectra_s * layer_nu,
        "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                       "kind": "one forward model, host call to device completion"},
        "kernel_ms": {"column": col_ms, "calls": n_timed,
                      "kind": "column kernel of timed steps 1, 9, 17, ... (counted from 0: every 8th from the second), from its launch's events"},
        "kernel_ms_breakdown": {"levels": ms_lev / max(n_break, 1),
                                "column": ms_col_b / max(n_break, 1),
                                "convolve_bin": ms_conv / max(n_break, 1), "calls": n_break,
                                "kind": "16 steps after the latency loop, before the warmup, every kernel timed"},
        "roofline": {
            "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
            "kernel": "k_column (fused opacity + short characteristics)",
            "algorithmic_bytes_per_launch": alg_bytes, "distinct_rows_per_species": U,
            "distinct_cia_rows": U_cia, "kernel_source": khash,
        },
        "valu_roof": valu,
    }
    if valu is not None:
        # the binding roof: the larger of the kernel's HBM time at the peak
        # (measured traffic when the counters match, else algorithmic bytes)
        # and its VALU issue time, against the measured kernel time
        hbm_us = (traffic if traffic else alg_bytes) / (HBM_PEAK_GBS * 1e9) * 1e6
        valu_us = valu["valu_issue_us"]
        roof_us = max(hbm_us, valu_us)
        res["binding_roof"] = {"hbm_us": hbm_us, "valu_issue_us": valu_us,
                               "bound": "valu" if valu_us >= hbm_us else "hbm",
                               "kernel_us": col_ms * 1e3, "frac": roof_us / (col_ms * 1e3)}
    if comparison is not None:
        res["comparison"] = comparison
    if not args.no_cpu_baseline:
        log("timing the oracle on the host")
        res["cpu_baseline"] = cpu_baseline(tab, cols[0], spec, n_mu, args.cpu_budget_s)
    print(json.dumps(res))


def run_oracle_timing(args):
    """The FP64 oracle timed on the host: per C1 and C2 spectrum with one thread
    and with all of them (median of 3; one single-threaded C2 run), and the
    C3 batch of 512 C1 sets.  Host-only; reports the core count and CPU."""
    import oracle
    import workloads as wl
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    all_threads = oracle.max_threads()

    def med(fn, reps):
        ts = []
        for _ in range(reps):
            t0 = time.perf_counter()
            fn()
            ts.append(time.perf_counter() - t0)
        return float(np.median(ts))

    res = {"workload": "FP64 oracle on the host", "cpu": model, "nproc": os.cpu_count(),
           "threads_all": all_threads}
    t1 = wl.c1_table()
    s1 = wl.c1_obs(t1)
    c1 = wl.c1_columns()[-1]
    f1 = lambda: oracle.forward(t1, c1, s1.window, s1.resolving_power, s1.edges_cm, 3)
    t2 = wl.c2_table(n_nu=args.n_nu)
    s2 = wl.c2_obs(t2)
    c2 = wl.c2_column()
    f2 = lambda: oracle.forward(t2, c2, s2.window, s2.resolving_power, s2.edges_cm, 3)
    c3 = wl.c3_columns()
    f3 = lambda: [oracle.forward(t1, c, s1.window, s1.resolving_power, s1.edges_cm, 3)
                  for c in c3]
    for n, tag in ((1, "1_thread"), (all_threads, "all_threads")):
        oracle.set_threads(n)
        log(f"oracle with {n} thread(s)")
        res[f"c1_s_per_spectrum_{tag}"] = med(f1, 3)
        res[f"c2_s_per_spectrum_{tag}"] = med(f2, 1 if n == 1 else 3)
        res[f"c3_s_per_batch_of_512_{tag}"] = med(f3, 1)
    oracle.set_threads(all_threads)
    # C5: the first 20 requests of the 2000 req/s serving trace, every set
    # (FP64 source table, all threads), as layer-nu points per second
    trace = wl.c5_trace_packed(t2, rate_hz=2000.0, duration_s=10.0)[:20]
    log(f"oracle on the C5 sample: {sum(r.n_sets for r in trace)} sets of 20 requests")
    t0 = time.perf_counter()
    for r in trace:
        for i in range(r.n_sets):
            c = wl.Column(r.p[i], r.T[i], r.x[i], r.log_g[i], r.scale[i])
            oracle.forward(t2, c, r.obs.window, r.obs.resolving_power, r.obs.edges_cm, 3)
    el = time.perf_counter() - t0
    res["c5_sample_layer_nu_per_s_all_threads"] = sum(r.layer_nu for r in trace) / el
    res["c5_sample"] = {"requests": 20, "sets": sum(r.n_sets for r in trace),
                        "layer_nu": sum(r.layer_nu for r in trace), "seconds": el}
    print(json.dumps(res))


def _dev_columns(cols):
    import torch
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()
    return (dev(np.stack([c.p_bar for c in cols])), dev(np.stack([c.T_K for c in cols])),
            dev(np.stack([c.x for c in cols])), dev([c.log_g for c in cols]),
            dev([c.scale for c in cols]))


def run_c1(args):
    """C1: one plain FP64 forward model (1 absorber, 5 x 5 table, 2000 points,
    20 layers, 3 angles, 50 bins) per call, each call synchronised: the
    latency of one small spectrum, launches included.  Device columns (the
    device entry) and host columns (the host entry, the column upload
    included); bins stay on the device."""
    import torch
    import workloads as wl
    from paper_1910_01070_amd import hr2
    tab = wl.c1_table()
    spec = wl.c1_obs(tab)
    cols = wl.c1_columns()
    ctx = hr2.Context(0)
    T = hr2.Tables(ctx, tab, "f64")
    obs = hr2.Obs(ctx, T, spec.window, spec.resolving_power, spec.edges_cm)
    res = {}
    for c in cols[-1:]:
        p, Tk, x, lg, sc = _dev_columns([c])
        bins = torch.empty(obs.n_bins, dtype=torch.float64, device="cuda")
        for name, call in (
                ("device_entry", lambda: hr2.forward_batch_dev(ctx, T, obs, p, Tk, x, lg, sc, 3, bins)),
                ("host_entry", lambda: hr2.forward_batch(ctx, T, obs, [c], 3, bins))):
            for _ in range(args.warmup):
                call()
                torch.cuda.synchronize()
            dt = []
            for _ in range(args.steps):
                t0 = time.perf_counter()
                call()
                torch.cuda.synchronize()
                dt.append(time.perf_counter() - t0)
            dt = np.array(dt)
            res[name] = {"p50_ms": float(np.median(dt) * 1e3),
                         "p99_ms": float(np.percentile(dt, 99) * 1e3),
                         "spectra_per_s": float(1.0 / np.mean(dt))}
    layer_nu = (cols[-1].n_levels - 1) * spec.window.count
    print(json.dumps({
        "metric": METRIC, "value": res["device_entry"]["spectra_per_s"], "unit": "spectra/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": 1e3 / res["device_entry"]["spectra_per_s"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "C1 plain FP64 forward model: 1 absorber, 5 T x 5 log p table, "
                               "2000 points at 1 cm^-1, 20 layers, 3 angles, R=300, 50 bins; "
                               "one synchronous call per spectrum"},
        "layer_nu_points_per_s": layer_nu * res["device_entry"]["spectra_per_s"],
        "latency": res,
    }))


def run_c3(args):
    """512 C1 sets: one batched launch captured in a HIP graph and replayed,
    against 512 sequential one-set calls (each synchronised)."""
    import torch
    import workloads as wl
    from paper_1910_01070_amd import hr2
    tab = wl.c1_table()
    spec = wl.c1_obs(tab)
    cols = wl.c3_columns()
    B = len(cols)
    ctx = hr2.Context(0)
    ctx.set_option(hr2.OPT_CHUNKS, args.chunks)
    T = hr2.Tables(ctx, tab, "f32")
    obs = hr2.Obs(ctx, T, spec.window, spec.resolving_power, spec.edges_cm)
    p, Tk, x, lg, sc = _dev_columns(cols)
    bins = torch.empty(B * obs.n_bins, dtype=torch.float32, device="cuda")
    fplus = torch.empty(B * spec.window.count, dtype=torch.float32, device="cuda")
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        for _ in range(3):
            hr2.forward_batch_dev(ctx, T, obs, p, Tk, x, lg, sc, 3, bins, fplus, None, s)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=s):
            hr2.forward_batch_dev(ctx, T, obs, p, Tk, x, lg, sc, 3, bins, fplus, None, s)
    torch.cuda.synchronize()
    for _ in range(args.warmup):
        g.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        g.replay()
    torch.cuda.synchronize()
    t_graph = (time.perf_counter() - t0) / args.steps
    t0 = time.perf_counter()
    for _ in range(args.steps):
        hr2.forward_batch_dev(ctx, T, obs, p, Tk, x, lg, sc, 3, bins, fplus)
    torch.cuda.synchronize()
    t_eager = (time.perf_counter() - t0) / args.steps
    one = torch.empty(obs.n_bins, dtype=torch.float32, device="cuda")
    for c in cols[:16]:
        hr2.forward_batch(ctx, T, obs, [c], 3, one)
        torch.cuda.synchronize()
    t0 = time.perf_counter()
    for c in cols:
        hr2.forward_batch(ctx, T, obs, [c], 3, one)
        torch.cuda.synchronize()
    t_seq = time.perf_counter() - t0
    layer_nu = (cols[0].n_levels - 1) * spec.window.count
    print(json.dumps({
        "metric": METRIC, "value": B / t_graph, "unit": "spectra/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": t_graph * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "512 C1 sets (1 absorber, 5x5 table, 2000 points, 20 layers, "
                               "3 angles, R=300, 50 bins) per launch, HIP graph replay"},
        "layer_nu_points_per_s": B * layer_nu / t_graph,
        "eager_batch_spectra_per_s": B / t_eager,
        "sequential_512_calls_spectra_per_s": B / t_seq,
        "graph_speedup_vs_sequential": t_seq / t_graph,
    }))


def run_c4(args):
    """C2 columns in batches of 1, 64 and 512 with FP32, FP16 and BF16 tables;
    every spectrum of every batch against the FP64 oracle on the FP64 source
    table (per-spectrum max relative error over the 400 bins)."""
    import torch
    import oracle
    import workloads as wl
    from paper_1910_01070_amd import hr2
    tab = wl.c2_table(n_nu=args.n_nu)
    spec = wl.c2_obs(tab)
    ctx = hr2.Context(0)
    batches = (1, 64, 512)
    all_cols = wl.c4_columns(max(batches))   # every batch is a prefix of this list
    log(f"FP64 oracle on the source table: {len(all_cols)} spectra")
    t0 = time.perf_counter()
    refs = []
    for i, c in enumerate(all_cols):
        refs.append(oracle.forward(tab, c, spec.window, spec.resolving_power, spec.edges_cm,
                                   3)["bins"])
        if (i + 1) % 64 == 0:
            log(f"  {i + 1} spectra, {time.perf_counter() - t0:.0f} s")
    refs = np.array(refs)
    rows = []
    errors = {}
    for label, dt, offset in (("f32", "f32", "row"), ("f16", "f16", "row"),
                              ("bf16", "bf16", "row"), ("f16/species-offset", "f16", "species"),
                              ("bf16/species-offset", "bf16", "species")):
        T = hr2.Tables(ctx, tab, dt, offset)
        obs = hr2.Obs(ctx, T, spec.window, spec.resolving_power, spec.edges_cm)
        errors[label] = {}
        for B in batches:
            cols = all_cols[:B]
            p, Tk, x, lg, sc = _dev_columns(cols)
            bins = torch.empty(B * obs.n_bins, dtype=torch.float32, device="cuda")
            steps = max(3, min(args.steps, 2000 // B))
            for _ in range(2):
                hr2.forward_batch_dev(ctx, T, obs, p, Tk, x, lg, sc, 3, bins)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(steps):
                hr2.forward_batch_dev(ctx, T, obs, p, Tk, x, lg, sc, 3, bins)
            torch.cuda.synchronize()
            dt_s = (time.perf_counter() - t0) / steps
            got = bins.cpu().numpy().reshape(B, obs.n_bins).astype(np.float64)
            err = np.max(np.abs(got - refs[:B]) / np.abs(refs[:B]), axis=1)
            errors[label][str(B)] = [float(f"{e:.3e}") for e in err]
            layer_nu = (cols[0].n_levels - 1) * spec.window.count
            rows.append({"table": label, "batch": B, "ms_per_launch": dt_s * 1e3,
                         "spectra_per_s": B / dt_s, "layer_nu_per_s": B * layer_nu / dt_s,
                         "max_rel_err_vs_fp64_oracle": float(err.max()),
                         "median_rel_err_vs_fp64_oracle": float(np.median(err))})
            log(rows[-1])
            del p, Tk, x, lg, sc, bins
        obs.close()
        T.close()
    print(json.dumps({"workload": "C4 reduced precision (C2 columns, batches)", "rows": rows,
                      "per_spectrum_max_rel_err_vs_fp64_oracle": errors,
                      "error_kind": "max over the 400 bins of |GPU - oracle| / |oracle|, the "
                                    "oracle in FP64 on the FP64 source table"}))


def run_params(args):
    """Parameter vectors to ln L: the paper's free-chemistry retrieval set-up
    (three second-order elements, seven free mixing ratios, error inflation:
    18 parameters) on the C2 table, batches of 1, 64 and 512 vectors per call
    (hr2_forward_params_dev with ln L only: one double per set comes back)."""
    import torch
    import workloads as wl
    from paper_1910_01070_amd import hr2
    tab = wl.c2_table(n_nu=args.n_nu)
    spec = wl.c2_obs(tab)
    lay = wl.c2_param_layout(3, 2, with_eps=True)
    ctx = hr2.Context(0)
    T = hr2.Tables(ctx, tab, args.dtype)
    obs = hr2.Obs(ctx, T, spec.window, spec.resolving_power, spec.edges_cm)
    P = hr2.Params(ctx, T, lay)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()
    # observed data: the model of one vector plus 20%-of-median noise (only
    # the shape of the data matters for timing)
    th0 = wl.draw_theta(lay, 1, seed=7)
    b0 = torch.empty(obs.n_bins, dtype=torch.float32, device="cuda")
    hr2.forward_params_dev(ctx, T, obs, P, dev(th0), 3, b0)
    torch.cuda.synchronize()
    D, sigma = wl.noisy_data(b0.cpu().numpy().astype(np.float64), seed=8)
    obs.set_data(D, sigma)
    rows = []
    L = lay.n_levels
    for B in (1, 64, 512):
        th = wl.draw_theta(lay, B, seed=100 + B)
        th[:, -1] = np.log10(float(sigma[0]) ** 2)
        thd = dev(th)
        lnl = torch.empty(B, dtype=torch.float64, device="cuda")
        steps = max(5, min(args.steps, 4000 // B))
        for _ in range(3):
            hr2.forward_params_dev(ctx, T, obs, P, thd, 3, None, lnl)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            hr2.forward_params_dev(ctx, T, obs, P, thd, 3, None, lnl)
        torch.cuda.synchronize()
        dt_s = (time.perf_counter() - t0) / steps
        rows.append({"batch": B, "ms_per_call": dt_s * 1e3, "likelihoods_per_s": B / dt_s,
                     "layer_nu_per_s": B * (L - 1) * spec.window.count / dt_s,
                     "finite": int(torch.isfinite(lnl).sum())})
        log(rows[-1])
    print(json.dumps({"workload": "parameter vectors -> ln L: 18-parameter free-chemistry "
                                  "set-up (3 second-order elements, 7 free ratios, eps) on the "
                                  "C2 table, 101 levels, 400 bins",
                      "table_storage": args.dtype, "rows": rows}))


def _serve_trace(hr2, srv, trace):
    """Submit a trace at its arrival times, collect every result; returns
    (latencies, done times, submit times, failures, submit-loop end)."""
    import threading
    tickets = [None] * len(trace)
    lat, done_t, sub_t = [], [], []
    fails = [0]

    def collect():
        for i, rq in enumerate(trace):
            while tickets[i] is None:
                time.sleep(0.0002)
            st, _, info = srv.poll(tickets[i], rq.n_sets * rq.obs.n_bins, wait_s=600.0)
            if st != hr2.OK:
                fails[0] += 1
                continue
            lat.append(info.t_done - info.t_submit)
            done_t.append(info.t_done)
            sub_t.append(info.t_submit)

    th = threading.Thread(target=collect)
    th.start()
    t0 = time.perf_counter()
    for i, rq in enumerate(trace):
        while time.perf_counter() - t0 < rq.t_arrival:
            pass
        tickets[i] = srv.submit_packed(rq.obs.window, rq.obs.resolving_power, rq.obs.edges_cm,
                                       rq.p, rq.T, rq.x, rq.log_g, rq.scale)
    t_sub_end = time.perf_counter() - t0
    th.join()
    return np.array(lat), done_t, sub_t, fails[0], t_sub_end


def serve_leg(ctx, T16, tab, rate, duration, strided_frac=0.5):
    """One Poisson trace against a fresh server on resident reduced-precision
    tables; returns (row of results, trace)."""
    import workloads as wl
    from paper_1910_01070_amd import hr2
    trace = wl.c5_trace_packed(tab, rate_hz=rate, duration_s=duration, strided_frac=strided_frac)
    srv = hr2.Server(ctx, T16, 16 << 30, 512)
    r = trace[0]   # warm the kernels once
    t = srv.submit_packed(r.obs.window, r.obs.resolving_power, r.obs.edges_cm, r.p, r.T,
                          r.x, r.log_g, r.scale)
    srv.poll(t, r.n_sets * r.obs.n_bins, wait_s=60.0)
    lat, done_t, sub_t, fails, t_sub_end = _serve_trace(hr2, srv, trace)
    stats = srv.stats()
    srv.close()
    span = max(done_t) - min(sub_t)
    work = sum(rq.layer_nu for rq in trace)
    strided = sum(rq.layer_nu for rq in trace if rq.obs.window.stride > 1)
    row = {
        "rate_req_per_s": rate, "duration_s": duration, "requests": len(trace),
        "failed": fails, "offered_layer_nu_per_s": work / duration,
        "served_layer_nu_per_s": work / span,
        "served_requests_per_s": len(lat) / span,
        "latency_s": {"p50": float(np.percentile(lat, 50)),
                      "p99": float(np.percentile(lat, 99)), "kind": "arrival to done"},
        "drain_s_after_last_arrival": max(done_t) - min(sub_t) - t_sub_end,
        "steps": stats.steps, "max_admitted": stats.max_inflight,
        "peak_bytes": stats.peak_bytes, "strided_work_frac": strided / work}
    return row, trace


def plain_leg(ctx, T32, sample):
    """The plain FP32 path on the same requests: one request at a time, its
    layout built and its sets run in one synchronous hr2_forward_batch call."""
    import torch
    import workloads as wl
    from paper_1910_01070_amd import hr2
    lat = []
    t0 = time.perf_counter()
    for rq in sample:
        t1 = time.perf_counter()
        obs = hr2.Obs(ctx, T32, rq.obs.window, rq.obs.resolving_power, rq.obs.edges_cm)
        cols = [wl.Column(rq.p[i], rq.T[i], rq.x[i], rq.log_g[i], rq.scale[i])
                for i in range(rq.n_sets)]
        bins = torch.empty(rq.n_sets * obs.n_bins, dtype=torch.float32, device="cuda")
        hr2.forward_batch(ctx, T32, obs, cols, 3, bins)
        torch.cuda.synchronize()
        obs.close()
        lat.append(time.perf_counter() - t1)
    t_plain = time.perf_counter() - t0
    return {"requests": len(sample),
            "layer_nu_per_s": sum(rq.layer_nu for rq in sample) / t_plain,
            "requests_per_s": len(sample) / t_plain,
            "service_time_s": {"p50": float(np.percentile(lat, 50)),
                               "p99": float(np.percentile(lat, 99)),
                               "kind": "one request alone, layout build to bins on the host"}}


def run_c5(args):
    """Poisson arrivals of uneven requests against the FP16-table server;
    then the plain FP32 one-request-at-a-time path on a sample of them.
    With --rates, a sweep of arrival rates (one fresh server each) instead."""
    import workloads as wl
    from paper_1910_01070_amd import hr2
    tab = wl.c2_table(n_nu=args.n_nu)
    ctx = hr2.Context(0)
    T16 = hr2.Tables(ctx, tab, args.dtype if args.dtype != "f32" else "f16")
    rates = [float(v) for v in args.rates.split(",")] if args.rates else [args.rate]
    rows = []
    for rate in rates:
        log(f"trace at {rate:g} req/s for {args.duration:g} s")
        row, trace = serve_leg(ctx, T16, tab, rate, args.duration, args.strided_frac)
        rows.append(row)
        log(rows[-1])
    desc = ("C5 serving trace: Poisson arrivals, 50-200 layers, 20k-150k point windows at 0.1 or "
            "1 cm^-1, R 100-1000, 1-64 sets per request, FP16 tables resident")
    if args.rates:
        print(json.dumps({"workload": desc + f", {args.duration:g} s per rate",
                          "rate_sweep": rows}))
        return
    T32 = hr2.Tables(ctx, tab, "f32")
    plain = plain_leg(ctx, T32, trace[: min(len(trace), 200)])
    res = dict(rows[0])
    res["workload"] = desc + f", {args.rate:g} req/s for {args.duration:g} s"
    res["plain_fp32_one_at_a_time_layer_nu_per_s"] = plain["layer_nu_per_s"]
    res["plain_fp32_one_at_a_time"] = plain
    res["speedup_vs_plain_fp32"] = res["served_layer_nu_per_s"] / plain["layer_nu_per_s"]
    print(json.dumps(res))


def batch_leg(ctx, tables_by_dtype, tab, B, steps):
    """C4 batches: B C2 columns per launch on each table type; spectra/s."""
    import torch
    import workloads as wl
    from paper_1910_01070_amd import hr2
    spec = wl.c2_obs(tab)
    cols = wl.c4_columns(B)
    p, Tk, x, lg, sc = _dev_columns(cols)
    layer_nu = (cols[0].n_levels - 1) * spec.window.count
    out = {}
    for dt, T in tables_by_dtype.items():
        obs = hr2.Obs(ctx, T, spec.window, spec.resolving_power, spec.edges_cm)
        bins = torch.empty(B * obs.n_bins, dtype=torch.float32, device="cuda")
        for _ in range(2):
            hr2.forward_batch_dev(ctx, T, obs, p, Tk, x, lg, sc, 3, bins)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            hr2.forward_batch_dev(ctx, T, obs, p, Tk, x, lg, sc, 3, bins)
        torch.cuda.synchronize()
        dt_s = (time.perf_counter() - t0) / steps
        out[dt] = {"ms_per_launch": dt_s * 1e3, "spectra_per_s": B / dt_s,
                   "layer_nu_per_s": B * layer_nu / dt_s}
        obs.close()
    return out


def comparison_legs(ctx, T32, tab, args):
    """The comparison, on the same GPU and in the same run as the headline:
    the batched reduced-precision serving path (a short C5 trace on FP16 tables)
    against the plain FP32 path one request at a time on the same requests,
    and 64-set batches with FP32 vs FP16 tables."""
    from paper_1910_01070_amd import hr2
    T16 = hr2.Tables(ctx, tab, "f16")
    log(f"comparison: C5 trace at {args.cmp_rate:g} req/s for {args.cmp_duration:g} s, FP16 tables")
    serving, trace = serve_leg(ctx, T16, tab, args.cmp_rate, args.cmp_duration)
    log(serving)
    sample = trace[: min(len(trace), args.cmp_plain)]
    log(f"comparison: plain FP32 path on {len(sample)} of the same requests")
    plain = plain_leg(ctx, T32, sample)
    log(plain)
    log("comparison: 64-set batches, FP16 vs FP32 tables")
    batches = batch_leg(ctx, {"f16": T16, "f32": T32}, tab, 64, 10)
    log(batches)
    return T16, {
        "serving_fp16_continuous_batching": serving,
        "plain_fp32_one_request_at_a_time": plain,
        "serving_speedup_vs_plain_fp32": serving["served_layer_nu_per_s"] / plain["layer_nu_per_s"],
        "batch64": batches,
        "batch64_fp16_vs_fp32": batches["f16"]["spectra_per_s"] / batches["f32"]["spectra_per_s"],
        "workload": ("C5: Poisson arrivals of uneven requests (50-200 layers, 20k-150k point "
                     "windows at 0.1 or 1 cm^-1, R 100-1000, 1-64 sets), FP16 tables resident, "
                     "16 GB budget; plain path: the same requests' first ones, FP32 tables, "
                     "one synchronous hr2_forward_batch each; batch64: 64 C2 columns per launch"),
    }


if __name__ == "__main__":
    main()
