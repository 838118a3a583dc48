"""The library's HLL wave-speed table (host code, no GPU needed) against the
oracle's and against closed forms (Part III eq:riemann-HLL).

The two tables are computed independently: the oracle differentiates the
printed M1 flux by complex step and takes numpy's eigenvalues; the library
differentiates the division-free flux by hand and solves the quadratic left
after removing the double transverse eigenvalue.  Bar: 1e-12 (in units of c).
"""
import numpy as np
import pytest

import oracle


@pytest.fixture(scope="module")
def lib_tab():
    from paper_2302_12727_amd import rt
    try:
        rt.load_library()
    except OSError as e:  # pragma: no cover
        pytest.skip(f"library not built: {e}")
    return rt.hll_speed_table()


def test_shape_and_grid(lib_tab):
    from paper_2302_12727_amd import rt
    assert lib_tab.shape == (rt.RT_HLL_NF, rt.RT_HLL_NMU, 2)


def test_library_table_equals_oracle_table(lib_tab, orc):
    ref = oracle.hll_table(lib_tab.shape[0], lib_tab.shape[1])
    err = np.abs(lib_tab - ref).max()
    assert err < 1e-12, err


def test_library_table_along_the_flux(lib_tab):
    # mu = +-1: the longitudinal 1D M1 system, eigenvalues
    # (chi' +- sqrt(chi'^2 + 4 (chi - f chi'))) / 2 with chi the Eddington
    # factor and chi' = dchi/df, both written out here
    nf = lib_tab.shape[0]
    f = np.arange(1, nf - 1) / (nf - 1)
    s = np.sqrt(4 - 3 * f * f)
    chi = (3 + 4 * f * f) / (5 + 2 * s)
    d = (8 * f * (5 + 2 * s) + (3 + 4 * f * f) * 6 * f / s) / (5 + 2 * s) ** 2
    r = np.sqrt(d * d + 4 * (chi - f * d))
    lo, hi = (d - r) / 2, (d + r) / 2
    assert np.abs(lib_tab[1:-1, -1, 0] - lo).max() < 1e-12
    assert np.abs(lib_tab[1:-1, -1, 1] - hi).max() < 1e-12
    assert np.abs(lib_tab[1:-1, 0, 0] + hi).max() < 1e-12
    assert np.abs(lib_tab[1:-1, 0, 1] + lo).max() < 1e-12


def test_library_table_limits_and_symmetry(lib_tab):
    nmu = lib_tab.shape[1]
    mu = -1 + 2 * np.arange(nmu) / (nmu - 1)
    assert np.allclose(lib_tab[0, :, 0], -1 / np.sqrt(3), rtol=0, atol=1e-15)
    assert np.allclose(lib_tab[0, :, 1], 1 / np.sqrt(3), rtol=0, atol=1e-15)
    assert np.array_equal(lib_tab[-1, :, 0], mu) and np.array_equal(lib_tab[-1, :, 1], mu)
    assert np.abs(lib_tab[:, :, 0] + lib_tab[:, ::-1, 1]).max() < 1e-13
    assert (lib_tab[:, :, 0] <= lib_tab[:, :, 1]).all()
    assert np.abs(lib_tab).max() <= 1 + 1e-13
