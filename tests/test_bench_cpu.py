"""CPU checks of the bench's roofline numerator (the algorithmic bytes of the
column kernel): the distinct table rows and CIA rows that
bench.algorithmic_bytes counts for a column are exactly the rows the
oracle's opacity (the bilinear interpolation in T and log p of Sect. 2.3)
depends on.  Changing any counted row changes the oracle's opacity of that
column; changing any other row leaves it unchanged.  The byte total is the
rows times the window times the element size, plus the CIA rows and the F+
write."""
import numpy as np

import bench
import oracle
from tests import hr2_testutil as tu


def _opacity(tab, col, idx):
    return oracle.opacity(tab, col, idx)


def test_counted_rows_are_the_rows_the_opacity_reads():
    tab = tu.small_multi_table()
    col = tu.small_columns(tab, 1, seed=23, n_levels=41)[0]
    idx = np.array([0, 7, 400, 1500, 2999])
    total, n_rows, n_cia = bench.algorithmic_bytes(tab, [col], 4, tab.n_nu, 5)
    chi0 = _opacity(tab, col, idx)
    nT, nP = len(tab.T_K), len(tab.log10_p_bar)
    rows, cia_rows = set(), set()
    for iT in range(nT):
        for ip in range(nP):
            saved = tab.log10_sigma[:, iT, ip, :].copy()
            tab.log10_sigma[:, iT, ip, :] += 3.0
            if not np.array_equal(_opacity(tab, col, idx), chi0):
                rows.add((iT, ip))
            tab.log10_sigma[:, iT, ip, :] = saved
        saved = tab.log10_k_cia[:, iT, :].copy()
        tab.log10_k_cia[:, iT, :] += 3.0
        if not np.array_equal(_opacity(tab, col, idx), chi0):
            cia_rows.add(iT)
        tab.log10_k_cia[:, iT, :] = saved
    assert len(rows) == n_rows and len(cia_rows) == n_cia
    assert 0 < n_rows < nT * nP
    S = tab.n_species
    assert total == S * n_rows * tab.n_nu * 4 + tab.n_cia * n_cia * tab.n_nu * 4 + tab.n_nu * 4


def test_rows_of_several_sets_are_counted_once():
    tab = tu.small_multi_table()
    cols = tu.small_columns(tab, 3, seed=29, n_levels=41)
    _, n_all, c_all = bench.algorithmic_bytes(tab, cols, 2, 100, 5)
    sets = [bench.algorithmic_bytes(tab, [c], 2, 100, 5) for c in cols]
    assert max(s[1] for s in sets) <= n_all <= sum(s[1] for s in sets)
    assert max(s[2] for s in sets) <= c_all <= sum(s[2] for s in sets)
    # the same column twice reads no new row
    assert bench.algorithmic_bytes(tab, [cols[0]] * 2, 2, 100, 5)[1] == sets[0][1]
