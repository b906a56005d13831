"""Helpers shared by the tests: error metrics, the storage-format replica used
to feed the oracle the dequantised tables, and cached seeded inputs."""
from __future__ import annotations

import functools

import numpy as np

import workloads as wl

LOG2_10 = np.log2(10.0)


def max_rel_err(got, ref, floor_frac=1e-30):
    """Per-spectrum max |got - ref| / max(|ref|, floor_frac * max|ref|) and the
    number of floored points."""
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    floor = floor_frac * np.max(np.abs(ref))
    den = np.maximum(np.abs(ref), floor)
    return float(np.max(np.abs(got - ref) / den)), int(np.sum(np.abs(ref) < floor))


def dequantised(table: wl.Table, dtype: str, offset: str = "row") -> wl.Table:
    """The table as libhr2 stores it (include/hr2.h, hr2_tables_desc.dtype and
    offset_mode): per row y = log10(sigma) log2(10) - off, off = (min + max)/2
    of the row ('row') or of the whole species ('species'), rounded to the
    storage type, returned in log10 units for the oracle.  CIA rows keep
    per-row offsets in either mode."""

    def conv(a):
        y = a * LOG2_10
        if offset == "species":
            off = 0.5 * (y.min(axis=(1, 2, 3), keepdims=True) + y.max(axis=(1, 2, 3), keepdims=True))
        else:
            off = 0.5 * (y.min(axis=-1, keepdims=True) + y.max(axis=-1, keepdims=True))
        q = y - off
        if dtype == "f16":
            q = q.astype(np.float16).astype(np.float64)
        elif dtype == "bf16":
            f = q.astype(np.float32)
            u = f.view(np.uint32).astype(np.uint64)
            u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
            q = u.astype(np.uint32).view(np.float32).astype(np.float64)
        elif dtype == "f32":
            q = q.astype(np.float32).astype(np.float64)
        else:
            raise ValueError(dtype)
        return (q + off) / LOG2_10

    sig = conv(table.log10_sigma)
    cia = None
    if table.log10_k_cia is not None:
        y = table.log10_k_cia * LOG2_10
        off = 0.5 * (y.min(axis=-1, keepdims=True) + y.max(axis=-1, keepdims=True))
        cia = ((y - off).astype(np.float32).astype(np.float64) + off) / LOG2_10
    return wl.Table(T_K=table.T_K, log10_p_bar=table.log10_p_bar, nu0_cm=table.nu0_cm,
                    dnu_cm=table.dnu_cm, n_nu=table.n_nu, log10_sigma=np.ascontiguousarray(sig),
                    molar_mass=table.molar_mass, log10_k_cia=cia, he_h2_ratio=table.he_h2_ratio,
                    species=table.species)


@functools.lru_cache(maxsize=None)
def c1_table():
    return wl.c1_table()


@functools.lru_cache(maxsize=None)
def c2_table():
    return wl.c2_table()


@functools.lru_cache(maxsize=None)
def small_multi_table():
    """3 species + CIA on a 6 T x 5 p grid, 3000 points at 0.5 cm^-1: several
    tiles and a ragged tail, every code path of the opacity stage."""
    return wl.make_table(77, ["H2O", "CH4", "CO"], [200.0, 500.0, 900.0, 1400.0, 2000.0, 2800.0],
                         [-5.0, -3.0, -1.0, 1.0, 2.5], 2000.0, 0.5, 3000, n_lines=300,
                         bands=True, s_range=(1e-24, 1e-19), with_cia=True)


def small_columns(table, n, seed=5, n_levels=41):
    rng = np.random.default_rng(seed)
    cols = []
    for _ in range(n):
        p = wl.levels(n_levels, 2.3, -4.7)
        T1 = rng.uniform(1200.0, 2700.0)
        b = rng.uniform(0.55, 0.95, 4)
        T = wl.piecewise_knot_profile(p, T1, b)
        x = wl.log_uniform(rng, 1e-6, 1e-2, table.n_species)
        cols.append(wl.Column(p, T, x, float(rng.uniform(3.5, 6.0)),
                              wl.scale_factor(rng.uniform(0.1, 5.0))))
    return cols
