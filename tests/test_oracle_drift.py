"""Pins of the oracle's drift correction (Part III "Dealing With Particle
Drifts"): U(x + dx) = U(x) + grad U(x) . dx per component.

- on a linear field the least-squares gradient is exact (eq:gradient), so the
  moved state is the field at the new position, for particles whose
  neighbourhood does not wrap around the periodic box;
- no displacement, no change (bitwise);
- a state moved below E = 0 is emptied, counted and booked in the ledger.
"""
import numpy as np
import pytest

import oracle
import workloads


@pytest.fixture(scope="module")
def lattice(orc):
    x = workloads.jittered_lattice(12, 0.2, 51)
    geo = oracle.build_geometry(x)
    return x, geo


def linear_field(x, G):
    g = workloads.rng(52)
    a = g.uniform(2.0, 3.0, size=(G, 4))
    a[:, 1:] *= 0.1
    b = g.uniform(-0.5, 0.5, size=(G, 4, 3))
    return a[None] + np.einsum("gma,na->ngm", b, x - 0.5)


def test_linear_field_moves_exactly(lattice):
    x, geo = lattice
    G = 2
    U = linear_field(x, G)
    dx = workloads.rng(53).uniform(-0.02, 0.02, size=(x.shape[0], 3))
    out, counts, ledger = oracle.drift(geo, U, dx)
    # particles whose gradient neighbourhood does not wrap around the box
    rows = np.repeat(np.arange(x.shape[0]), np.diff(geo.gptr))
    wraps = np.abs(x[geo.gidx] - x[rows]).max(axis=1) > 0.5
    inner = np.ones(x.shape[0], dtype=bool)
    inner[rows[wraps]] = False
    assert inner.sum() > 100
    ref = linear_field(x + dx, G)
    err = np.abs(out - ref)[inner].max() / np.abs(ref).max()
    assert err < 1e-12
    assert not counts.any() and not ledger.any()


def test_no_displacement(lattice):
    x, geo = lattice
    U = linear_field(x, 1)
    out, _, _ = oracle.drift(geo, U, np.zeros((x.shape[0], 3)))
    assert np.array_equal(out, U)


def test_guard_and_ledger(lattice):
    x, geo = lattice
    n = x.shape[0]
    U = np.zeros((n, 1, 4))
    U[:, 0, 0] = 1.0
    dU = np.zeros((n, 1, 4, 3))
    dU[:, 0, 0, 0] = 10.0                   # dE/dx = 10
    dx = np.zeros((n, 3))
    dx[: n // 2, 0] = -0.2                   # E = 1 - 2 = -1 for the first half
    out, counts, ledger = oracle.drift(geo, U, dx, dU=dU)
    assert not out[: n // 2].any()
    assert np.array_equal(out[n // 2:], U[n // 2:])
    assert counts[2] == n // 2 and counts[3] == 0
    assert ledger[0] == pytest.approx(geo.V[: n // 2].sum(), rel=1e-13)
