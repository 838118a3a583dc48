"""Pins of the oracle's photo-absorption (Part III "Third step:
Thermochemistry") and of its photon-group constants (Part III "Discretization
of Frequencies", eq:sigma-parametrizaiton with tab:cross-sections,
eq:blackbody).

- group luminosities against the values the thesis prints for its Iliev
  Test 2 source (tests/golden/group_luminosities.txt; 1, 3 and 10 groups);
- cross sections: textbook threshold values, the hydrogenic scaling of He+
  against H, the E^-3.5 fall-off far above threshold, zero below threshold;
- group averages against an independent composite-trapezoid quadrature, the
  narrow-group limit, zero for species whose threshold lies above the group;
- the removal: forward Euler converges to the exact solution exp(-c kappa t)
  of eq:thermochemistry-E/F at first order; the step-averaged densities; the
  photon budget; E and F scaled alike; the clamp; no absorber, no change.
"""
import os

import numpy as np
import pytest

import oracle
import workloads
from oracle import photons

GOLD = os.path.join(os.path.dirname(__file__), "golden", "group_luminosities.txt")


def golden_runs():
    runs = {}
    for line in open(GOLD):
        if line.startswith("#") or not line.strip():
            continue
        run, _, lo, hi, L = line.split()
        runs.setdefault(run, []).append((float(lo), float(hi), float(L)))
    return runs


@pytest.mark.parametrize("run", ["g1", "g3", "g10"])
def test_group_luminosities_as_printed(run):
    rows = golden_runs()[run]
    edges = [r[0] for r in rows] + [rows[-1][1]]
    L = photons.group_luminosities(edges, 1e5, 5e48) / photons.L_SOL
    ref = np.array([r[2] for r in rows])
    # 4 printed digits and the solar luminosity's convention: 1e-3
    assert np.abs(L / ref - 1).max() < 1e-3
    assert np.abs((L / L.sum()) / (ref / ref.sum()) - 1).max() < 1e-3


def test_cross_sections_at_threshold_and_below():
    s = [float(photons.cross_section(j, photons.E_ION[j])) for j in range(3)]
    assert s[0] == pytest.approx(6.30e-18, rel=0.01)     # H0
    assert s[1] == pytest.approx(7.43e-18, rel=0.01)     # He0
    assert s[2] == pytest.approx(1.58e-18, rel=0.01)     # He+
    for j in range(3):
        assert photons.cross_section(j, photons.E_ION[j] * (1 - 1e-9)) == 0.0


def test_he_plus_is_hydrogenic():
    # a hydrogen-like ion of charge Z has sigma_Z(Z^2 E) = sigma_H(E) / Z^2;
    # the two fits agree with that to their printed digits
    E = np.geomspace(13.7, 1e4, 50)
    r = photons.cross_section(2, 4 * E) / (photons.cross_section(0, E) / 4)
    assert np.abs(r - 1).max() < 3e-3


def test_fall_off_far_above_threshold():
    for j in range(3):
        E = 1e7
        slope = np.log(photons.cross_section(j, 1.01 * E) / photons.cross_section(j, E)) / np.log(1.01)
        assert abs(slope + 3.5) < 0.01


def test_group_averages_against_trapezoid():
    edges = [13.6, 24.59, 54.42, np.inf]
    T = 1e5
    sN, sE, eps, frac = photons.group_constants(edges, T)
    kT = photons.K_B * T / photons.EV
    tot_n = 0.0
    for i in range(3):
        a = edges[i]
        b = edges[i + 1] if np.isfinite(edges[i + 1]) else a + 90 * kT
        E = np.linspace(a, b, 400001)
        wn = E ** 2 / np.expm1(E / kT)
        we = E ** 3 / np.expm1(E / kT)
        n_i, e_i = np.trapezoid(wn, E), np.trapezoid(we, E)
        tot_n += n_i
        assert eps[i] / photons.EV == pytest.approx(e_i / n_i, rel=1e-8)
        for j in range(3):
            # the group is [a, b): a species whose threshold is b absorbs nothing
            s = photons.cross_section(j, E) if photons.E_ION[j] < b else np.zeros_like(E)
            assert sN[i, j] == pytest.approx(np.trapezoid(wn * s, E) / n_i, rel=1e-7, abs=1e-30)
            assert sE[i, j] == pytest.approx(np.trapezoid(we * s, E) / e_i, rel=1e-7, abs=1e-30)
    # thresholds at the group edges: no species absorbs below its threshold
    assert sN[0, 1] == 0 and sN[0, 2] == 0 and sN[1, 2] == 0
    assert np.abs(frac.sum() - 1) < 1e-12
    assert (eps / photons.EV >= np.array(edges[:-1])).all()


def test_narrow_group_is_the_cross_section():
    sN, sE, eps, _ = photons.group_constants([30.0, 30.001], 1e5)
    s = photons.cross_section(0, 30.0005)
    assert sN[0, 0] == pytest.approx(s, rel=1e-7)
    assert sE[0, 0] == pytest.approx(s, rel=1e-7)
    assert eps[0] / photons.EV == pytest.approx(30.0005, rel=1e-7)


@pytest.fixture(scope="module")
def small(orc):
    w = workloads.lattice_workload(8, 2, 0, 1, seed=61, name="absorb")
    geo = oracle.build_geometry(w.x)
    g = workloads.rng(62)
    n_old = g.uniform(0.0, 1.0, size=(w.n, 3))
    n_new = n_old * g.uniform(0.2, 1.0, size=(w.n, 3))      # the gas ionizes
    sigma = np.array([[0.30, 0.0, 0.0], [0.06, 0.45, 0.0]])
    return w, geo, n_old, n_new, sigma


def test_euler_converges_to_the_exponential(small):
    w, geo, n_old, _, sigma = small
    t = 0.8
    kappa = n_old @ sigma.T                              # [n][G]
    exact = w.U0 * np.exp(-geo.c * kappa * t)[..., None]
    errs = []
    for m in (8, 16, 32, 64):
        U = w.U0.copy()
        for _ in range(m):
            U, _ = oracle.absorb(geo, U, n_old, sigma, t / m)
        err = np.abs(U - exact).max(axis=-1) / np.abs(w.U0).max(axis=-1)
        bound = (geo.c * kappa * t) ** 2 / (2 * m)
        assert (err <= bound * 1.0001 + 1e-15).all()
        errs.append(err.max())
    ratios = np.array(errs[:-1]) / np.array(errs[1:])
    assert np.abs(ratios - 2).max() < 0.1                # first order


def test_densities_averaged_over_the_step(small):
    w, geo, n_old, n_new, sigma = small
    got, _ = oracle.absorb(geo, w.U0, n_old, sigma, 0.3, n_new=n_new)
    ref, _ = oracle.absorb(geo, w.U0, 0.5 * (n_old + n_new), sigma, 0.3)
    assert np.abs(got - ref).max() <= 1e-15 * np.abs(w.U0).max()
    old, _ = oracle.absorb(geo, w.U0, n_old, sigma, 0.3)
    assert np.abs(got - old).max() > 1e-3 * np.abs(w.U0).max()


def test_budget_and_direction(small):
    w, geo, n_old, n_new, sigma = small
    got, absorbed = oracle.absorb(geo, w.U0, n_old, sigma, 0.5, n_new=n_new)
    Q0, Q1 = oracle.photon_total(geo, w.U0), oracle.photon_total(geo, got)
    assert np.abs((Q0 - Q1) / absorbed - 1).max() < 1e-12
    assert (absorbed > 0).all()
    # E and F scaled by the same factor: reduced flux and direction kept
    ratio = got[..., 1:] / got[..., :1]
    assert np.abs(ratio - w.U0[..., 1:] / w.U0[..., :1]).max() < 1e-13 * np.abs(ratio).max()


def test_clamp_and_no_absorber(small):
    w, geo, n_old, _, sigma = small
    got, absorbed = oracle.absorb(geo, w.U0, 1e6 * n_old + 1.0, sigma, 1.0)
    assert not got.any()
    assert np.allclose(absorbed, oracle.photon_total(geo, w.U0), rtol=1e-13)
    same, absorbed0 = oracle.absorb(geo, w.U0, np.zeros_like(n_old), sigma, 1.0)
    assert np.array_equal(same, w.U0) and not absorbed0.any()
