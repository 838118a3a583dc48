"""Pins of the oracle's global time step (Part III eq:rt-cfl with one global
step): dt = C_cfl min_i dx_i / c, dx_i = (3 V_i / 4 pi)^{1/3} the radius of
the sphere of the particle's volume.

- Perfect lattices of spacing d: the volume of a particle is d^3 up to the
  lattice sum of the kernel, so dt = C_cfl (3 / 4 pi)^{1/3} d / c to 2e-3,
  with one and the same ratio for every spacing, box size, c and C_cfl (a
  4 pi in place of 4 pi / 3 is 44% off, a factor 2 is 100% off).
- Solved smoothing lengths: the h equation with the self term,
  h^3 sum_j W(r_ij, kappa h) = eta^3 (eq:number-of-neighbors), and
  V = 1/omega (eq:particle-volume) give V_i = (h_i / eta)^3, so
  dt = C_cfl (3 / 4 pi)^{1/3} min_i h_i / (eta c) to the solver's tolerance on
  a jittered lattice and on a clustered set: the step is tied to the
  smoothing lengths, which the brute-force residual test pins.
"""
import numpy as np
import pytest

import oracle
import workloads

CUBE = (3.0 / (4.0 * np.pi)) ** (1.0 / 3.0)


def test_perfect_lattice_closed_form(orc):
    ratios = []
    for n_side, box, c, cfl in ((10, 1.0, 1.0, 0.9), (14, 1.0, 2.5, 0.3), (12, 2.0, 1.0, 0.9),
                                (12, 1.0, 0.4, 0.6)):
        x = workloads.perfect_lattice(n_side) * box
        geo = oracle.build_geometry(x, c=c, cfl=cfl, box=box)
        d = box / n_side
        r = geo.dt / (cfl * CUBE * d / c)
        ratios.append(r)
        assert abs(r - 1) < 2e-3, (n_side, box, c, cfl, r)
    assert np.ptp(ratios) < 1e-12 * np.mean(ratios)


@pytest.mark.parametrize("kind", ["lattice", "plummer"])
def test_step_follows_the_smallest_smoothing_length(orc, kind):
    if kind == "lattice":
        x = workloads.jittered_lattice(11, 0.1, 21)
    else:
        x = workloads.plummer_mix(3000, 0.05, 0.5, 0.1, seed=22)
    for c, cfl in ((1.0, 0.9), (3.0, 0.5)):
        geo = oracle.build_geometry(x, c=c, cfl=cfl)
        # V_i = (h_i / eta)^3 particle by particle
        assert np.abs(geo.V / (geo.h / geo.eta) ** 3 - 1).max() < 1e-12
        ref = cfl * CUBE * geo.h.min() / (geo.eta * c)
        assert abs(geo.dt / ref - 1) < 1e-12
