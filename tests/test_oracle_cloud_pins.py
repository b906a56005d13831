"""Pins of the gray cloud layer in the oracle (App. B): how its optical depth
is spread over the layers (worked by hand under the reading "uniform in
ln p"), and the emergent flux in limits with closed forms: an opaque cloud
under a transparent atmosphere emits pi B(T at the cloud top), an isothermal
column emits pi B(T) whatever the cloud, and a cloud of zero optical depth
changes nothing."""
import numpy as np
import pytest

import oracle


def test_cloud_share_by_hand():
    p = np.array([100.0, 10.0, 1.0, 0.1])
    # top 1 bar, bottom 100 bar: the two lower layers each cover half of ln p
    d = oracle.cloud_dtau(p, (8.0, 1.0, 100.0))
    assert np.allclose(d, [4.0, 4.0, 0.0], rtol=1e-15, atol=0)
    # top 3 bar, bottom 30 bar: layer 0 holds [ln 10, ln 30], layer 1 [ln 3, ln 10]
    d = oracle.cloud_dtau(p, (1.0, 3.0, 10.0))
    assert np.allclose(d, [np.log(3.0) / np.log(10.0), np.log(10.0 / 3.0) / np.log(10.0), 0.0],
                       rtol=1e-14, atol=0)
    assert abs(d.sum() - 1.0) < 1e-15
    # a cloud reaching below the column's bottom keeps only the part inside
    d = oracle.cloud_dtau(p, (2.0, 10.0, 100.0))      # 10 .. 1000 bar: half is inside
    assert np.allclose(d, [1.0, 0.0, 0.0], rtol=1e-15, atol=0)
    assert np.all(oracle.cloud_dtau(p, (0.0, 1.0, 100.0)) == 0.0)


def _column(L=30):
    p = 10.0 ** np.linspace(2.0, -4.0, L)
    T = 2200.0 - 900.0 * np.linspace(0.0, 1.0, L) ** 0.7
    dz = np.full(L - 1, 1.0e6)
    return p, T, dz


@pytest.mark.parametrize("k", [5, 12, 29])
def test_opaque_cloud_under_a_transparent_gas_emits_the_top_level(k):
    p, T, dz = _column()
    nu = np.array([500.0, 2000.0, 7000.0])
    chi = np.zeros((len(p), len(nu)))
    ext = oracle.cloud_dtau(p, (1.0e15, p[k], 1.0e3))
    F = oracle.rt_emission(chi, dz, T, nu, 3, ext)
    want = np.pi * oracle.planck(nu, np.full(3, T[k]))
    assert np.allclose(F, want, rtol=1e-12, atol=0)


def test_isothermal_column_ignores_the_cloud():
    p, _, dz = _column()
    T = np.full(len(p), 1500.0)
    nu = np.array([800.0, 4000.0])
    rng = np.random.default_rng(3)
    chi = 10.0 ** rng.uniform(-9, -5, (len(p), 2))
    for cloud in ((0.3, 0.5, 4.0), (40.0, 1e-3, 1e4)):
        F = oracle.rt_emission(chi, dz, T, nu, 4, oracle.cloud_dtau(p, cloud))
        assert np.allclose(F, np.pi * oracle.planck(nu, np.full(2, 1500.0)), rtol=1e-13)


def test_zero_cloud_is_clear_sky():
    p, T, dz = _column()
    nu = np.array([600.0, 3000.0])
    rng = np.random.default_rng(4)
    chi = 10.0 ** rng.uniform(-9, -5, (len(p), 2))
    a = oracle.rt_emission(chi, dz, T, nu, 3)
    b = oracle.rt_emission(chi, dz, T, nu, 3, oracle.cloud_dtau(p, (0.0, 1.0, 10.0)))
    assert np.array_equal(a, b)
    # and a thick cloud deep in a cooling column dims the emission
    c = oracle.rt_emission(chi, dz, T, nu, 3, oracle.cloud_dtau(p, (50.0, 1.0, 10.0)))
    assert np.all(c < a)
