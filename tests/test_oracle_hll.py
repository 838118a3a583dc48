"""Pins of the oracle's HLL solver (Part III eq:riemann-HLL) and of its
eigenvalue table.

- table at mu = cos(theta) = +-1 against the closed form of the 1D M1 system
  (the longitudinal 2x2 Jacobian [[0, 1], [c^2 (chi - f chi'), c chi']] has
  eigenvalues c (chi' +- sqrt(chi'^2 + 4 (chi - f chi'))) / 2), differentiated
  by hand here, independently of the complex-step Jacobian;
- f = 0 nodes at -+1/sqrt(3); mirror symmetry l_min(f, mu) = -l_max(f, -mu);
  |l| <= 1 (no signal faster than c);
- interior nodes against the spectrum of the flux Jacobian at random 3D
  orientations, energies and speeds of light (rotation and scale
  invariance), which must also hold the closed-form transverse mode;
- HLL with wave speeds -+c is the GLF solver (the thesis states it); a
  two-identical-state Riemann problem returns the state's flux; with both
  speeds positive the flux is the upwind one;
- one HLL transport step conserves photons (no sources; the face guards act
  on the same face states from both sides of a pair, so only the post-update
  guard, which does not fire here, could change the total).
"""
import numpy as np
import pytest

import oracle
import workloads


@pytest.fixture(scope="module")
def tab(orc):
    return oracle.hll_table()


def chi_and_slope(f):
    s = np.sqrt(4 - 3 * f * f)
    chi = (3 + 4 * f * f) / (5 + 2 * s)
    dchi = (8 * f * (5 + 2 * s) + (3 + 4 * f * f) * 6 * f / s) / (5 + 2 * s) ** 2
    return chi, dchi


def test_table_along_the_flux_is_the_1d_system(tab):
    nf, nmu = tab.shape[:2]
    worst = 0.0
    for i in range(1, nf - 1):
        f = i / (nf - 1)
        chi, d = chi_and_slope(f)
        r = np.sqrt(d * d + 4 * (chi - f * d))
        lo, hi = (d - r) / 2, (d + r) / 2
        worst = max(worst, abs(tab[i, -1, 0] - lo), abs(tab[i, -1, 1] - hi))
        worst = max(worst, abs(tab[i, 0, 0] + hi), abs(tab[i, 0, 1] + lo))
    assert worst < 1e-12


def test_table_limits_symmetry_and_bounds(tab):
    assert np.allclose(tab[0, :, 0], -1 / np.sqrt(3), rtol=0, atol=1e-15)
    assert np.allclose(tab[0, :, 1], 1 / np.sqrt(3), rtol=0, atol=1e-15)
    assert np.abs(tab[:, :, 0] + tab[:, ::-1, 1]).max() < 1e-13
    assert (tab[:, :, 0] <= tab[:, :, 1] + 1e-15).all()
    assert np.abs(tab).max() <= 1 + 1e-13


def rotation(g):
    """A random proper rotation (QR of a Gaussian matrix, signs fixed)."""
    q, r = np.linalg.qr(g.normal(size=(3, 3)))
    q = q * np.sign(np.diag(r))
    return q if np.linalg.det(q) > 0 else -q


def test_table_interior_by_rotation_and_the_transverse_mode(tab):
    """Interior nodes 0 < f < 1, -1 < mu < 1.  The table is built at one
    orientation (F along x, the normal in the x-y plane, E = 1, c = 1); here
    the flux Jacobian d(F.n, c^2 P n)/d(E, F) of the printed closure is taken
    at a random 3D orientation, a random energy and c != 1 with |F| = c f E
    and F.n = mu |F|.  Its eigenvalues divided by c must have the table's
    extremes at that node, and one of them must be the transverse mode
    3 f mu / (2 + sqrt(4 - 3 f^2)): a perturbation dF normal to the plane of F
    and n keeps f and chi, turns F/|F| by dF/|F|, and so changes c^2 P n by
    c^2 E (3 chi - 1)/2 mu dF / |F| = c mu (3 chi - 1)/(2 f) dF, which the
    identity (3 chi - 1)/(2 f^2) = 3/(2 + sqrt(4 - 3 f^2)) turns into the
    closed form.  A wrong mu -> n mapping of the table, or wrong units, fails."""
    g = workloads.rng(41)
    nf, nmu = tab.shape[:2]
    hstep = 1e-30
    for _ in range(80):
        i, j = int(g.integers(1, nf - 1)), int(g.integers(1, nmu - 1))
        f, mu = i / (nf - 1), -1.0 + 2.0 * j / (nmu - 1)
        c = float(g.choice([1.0, 2.5, 0.3]))
        E = float(g.lognormal())
        R = rotation(g)
        d_F, d_p, d_t = R[:, 0], R[:, 1], R[:, 2]
        n = mu * d_F + np.sqrt(1.0 - mu * mu) * d_p
        U = np.concatenate([[E], c * f * E * d_F])
        J = np.zeros((4, 4))
        for k in range(4):
            Uc = U.astype(complex)
            Uc[k] += 1j * hstep
            J[:, k] = oracle.m1_flux_printed(Uc, n, c).imag / hstep
        ev = np.linalg.eigvals(J)
        assert np.abs(ev.imag).max() < 1e-8 * c
        lam = np.sort(ev.real) / c
        assert abs(lam[0] - tab[i, j, 0]) < 1e-11 and abs(lam[-1] - tab[i, j, 1]) < 1e-11
        mt = 3.0 * f * mu / (2.0 + np.sqrt(4.0 - 3.0 * f * f))
        assert np.abs(lam - mt).min() < 1e-11
        v = np.concatenate([[0.0], d_t])
        assert np.linalg.norm(J @ v - c * mt * v) < 1e-11 * c


def random_state(g, f):
    E = g.lognormal()
    d = g.normal(size=3)
    d /= np.linalg.norm(d)
    return np.concatenate([[E], f * E * d])


def test_hll_with_speed_of_light_is_glf(orc):
    g = workloads.rng(31)
    box = np.full((2, 2, 2), -1.0)
    box[..., 1] = 1.0
    for _ in range(50):
        qL, qR = random_state(g, g.uniform()), random_state(g, g.uniform())
        nh = g.normal(size=3)
        nh /= np.linalg.norm(nh)
        ref = np.zeros(4)
        oracle.lib().orc_glf(oracle._p(qL), oracle._p(qR), oracle._p(nh), 1.0, oracle._p(ref))
        got = oracle.hll_flux(qL, qR, nh, box)
        assert np.abs(got - ref).max() <= 1e-14 * np.abs(ref).max()


def test_hll_consistency_and_upwinding(tab):
    g = workloads.rng(32)
    for _ in range(50):
        q = random_state(g, g.uniform())
        nh = g.normal(size=3)
        nh /= np.linalg.norm(nh)
        fl = np.zeros(4)
        oracle.lib().orc_m1_flux(oracle._p(q), oracle._p(nh), 1.0, oracle._p(fl))
        got = oracle.hll_flux(q, q, nh, tab)
        assert np.abs(got - fl).max() <= 1e-14 * np.abs(fl).max() + 1e-300
    # nearly free streaming along the normal: both wave speeds positive
    nh = np.array([1.0, 0.0, 0.0])
    qL = np.array([1.0, 0.995, 0.0, 0.0])
    qR = np.array([2.0, 1.98, 0.05, 0.0])
    fl = np.zeros(4)
    oracle.lib().orc_m1_flux(oracle._p(qL), oracle._p(nh), 1.0, oracle._p(fl))
    assert np.array_equal(oracle.hll_flux(qL, qR, nh, tab), fl)


def test_hll_step_conserves_photons(tab):
    w = workloads.lattice_workload(10, 2, 0, 1, seed=77, name="hll")
    U0 = w.U0.copy()
    U0[..., 1:] *= 0.3        # far from the free-streaming limit
    geo = oracle.build_geometry(w.x)
    out, info = oracle.step(geo, None, U0, hll=tab)
    assert not info["counts"][2:].any()       # the post-update guard did not fire
    Q0, Q1 = oracle.photon_total(geo, U0), oracle.photon_total(geo, out)
    assert np.abs(Q1 / Q0 - 1).max() < 1e-13
    glf, _ = oracle.step(geo, None, U0)
    assert np.abs(out - glf).max() > 1e-6 * np.abs(glf).max()   # a different solver


def test_binned_hll_reduces_to_the_global_step(tab):
    # individual time steps with every particle in bin 0 are the global step,
    # and with every particle in bin 1 two ticks are one global step of 2 dt
    w = workloads.lattice_workload(9, 2, 2, 3, seed=78, name="hllbins")
    geo = oracle.build_geometry(w.x)
    srcs = oracle.build_sources(geo, w.xs)
    def state_err(got, ref):      # per state, floored for states a guard emptied
        scale = np.maximum(np.abs(ref).max(axis=-1), 1e-6 * np.abs(ref[..., 0]).mean())
        return float((np.abs(got - ref).max(axis=-1) / scale).max())

    ref, _ = oracle.run(geo, srcs, w.U0, w.L, 3, hll=tab)
    got, info = oracle.run_binned(geo, srcs, w.U0, w.L, 3, np.zeros(geo.n, np.int32), hll=tab)
    assert state_err(got, ref) < 1e-12
    assert not info["acc"].any()
    ref2, _ = oracle.step(geo, srcs, w.U0, w.L, dt=2.0 * geo.dt, hll=tab)
    got2, _ = oracle.run_binned(geo, srcs, w.U0, w.L, 2, np.ones(geo.n, np.int32), hll=tab)
    assert state_err(got2, ref2) < 1e-12
    glf, _ = oracle.run_binned(geo, srcs, w.U0, w.L, 3, np.zeros(geo.n, np.int32))
    assert np.abs(glf - got).max() > 1e-6 * np.abs(got).max()
