"""Photon-group constants for photo-absorption -- TEST INFRASTRUCTURE ONLY
(part of the oracle; only tests/, the smoke check and the CPU-baseline leg of
bench.py may import it).

Written from the thesis (arXiv:2302.12727), Part III:
  * photo-ionization cross sections of H0, He0, He+ from the analytic fits of
    eq:sigma-parametrizaiton with the parameters of tab:cross-sections; zero
    below each species' ionization energy (eq:nuIonHI - eq:nuIonHeII);
  * the blackbody spectrum eq:blackbody;
  * group averages over a frequency group i: the number-weighted cross section
    sigma^N_ij (eq:sigma_N), the energy-weighted sigma^E_ij (same section) and
    the mean photon energy eps_i = int J / int J/(h nu);
  * the conversion of a photon number rate into group luminosities, appendix
    "Converting Photon Number Emission Rates to Photon Energy Emission Rates":
    L_i = Ndot int_i J / int_{nu_min}^inf J/(h nu).

Reading: tab:cross-sections lists sigma_0 already in cm^2 (the Verner fits'
sigma_0 in Mb times 1e-18), so sigma(E) = sigma_0 F(y) with that value; the
extra factor 1e-18 of the printed formula would apply to sigma_0 in Mb.

Integrals: scipy.integrate.quad (a library primitive) in the variable
x = E / (k_B T), split at the species thresholds inside a group.
"""
from __future__ import annotations

import numpy as np
from scipy.integrate import quad

# physical constants (cgs; h and k_B exact in SI 2019, eV exact)
H_PLANCK = 6.62607015e-27     # erg s
K_B = 1.380649e-16            # erg / K
EV = 1.602176634e-12          # erg
L_SOL = 3.828e33              # erg / s (IAU 2015 nominal solar luminosity)

SPECIES = ("HI", "HeI", "HeII")
# ionization energies in eV (eq:nuIonHI, eq:nuIonHeI, eq:nuIonHeII)
E_ION = np.array([13.60, 24.59, 54.42])
# tab:cross-sections: E_0 [eV], sigma_0 [cm^2], y_a, P, y_w, y_0, y_1
VERNER = np.array([
    [0.4298, 5.475e-14, 32.88, 2.963, 0.0, 0.0, 0.0],
    [13.61, 9.492e-16, 1.469, 3.188, 2.039, 0.4434, 2.136],
    [1.720, 1.369e-14, 32.88, 2.963, 0.0, 0.0, 0.0],
])


def cross_section(j: int, E_eV) -> np.ndarray:
    """sigma_j(E) in cm^2 for photon energies E in eV (eq:sigma-parametrizaiton),
    0 below the ionization energy of species j."""
    E = np.asarray(E_eV, dtype=np.float64)
    E0, s0, ya, P, yw, y0, y1 = VERNER[j]
    x = E / E0 - y0
    y = np.sqrt(x * x + y1 * y1)
    F = ((x - 1.0) ** 2 + yw * yw) * y ** (0.5 * P - 5.5) * (1.0 + np.sqrt(y / ya)) ** (-P)
    return np.where(E >= E_ION[j], s0 * F, 0.0)


def _integral(fn, a: float, b: float, breaks=()) -> float:
    pts = [a] + sorted(p for p in breaks if a < p < b) + [b]
    tot = 0.0
    for lo, hi in zip(pts[:-1], pts[1:]):
        tot += quad(fn, lo, hi, epsabs=0.0, epsrel=1e-13, limit=400)[0]
    return tot


def group_constants(edges_eV, T_bb: float):
    """Group averages for a blackbody of temperature T_bb (K) over the groups
    [edges_eV[i], edges_eV[i+1]) (the last edge may be inf).

    Returns (sigma_N [G][3] cm^2, sigma_E [G][3] cm^2, eps [G] erg,
    frac [G]): frac_i = int_i J/(h nu) / int_{edges[0]}^inf J/(h nu), the
    fraction of the photons above the first edge that fall in group i."""
    kT_eV = K_B * T_bb / EV
    xe = [e / kT_eV for e in edges_eV]
    xi = E_ION / kT_eV
    # spectrum in x = h nu / kT: J dnu ~ x^3/(e^x - 1) dx, photon number
    # ~ x^2/(e^x - 1) dx, written with e^-x so that large x does not overflow
    num = lambda x: x * x * np.exp(-x) / -np.expm1(-x)
    eng = lambda x: x ** 3 * np.exp(-x) / -np.expm1(-x)
    G = len(edges_eV) - 1
    sN = np.zeros((G, 3))
    sE = np.zeros((G, 3))
    eps = np.zeros(G)
    frac = np.zeros(G)
    n_all = _integral(num, xe[0], np.inf)
    for i in range(G):
        a, b = xe[i], xe[i + 1]
        n_i = _integral(num, a, b)
        e_i = _integral(eng, a, b)
        eps[i] = e_i / n_i * K_B * T_bb
        frac[i] = n_i / n_all
        for j in range(3):
            sig = lambda x, j=j: float(cross_section(j, x * kT_eV))
            sN[i, j] = _integral(lambda x: num(x) * sig(x), a, b, xi) / n_i
            sE[i, j] = _integral(lambda x: eng(x) * sig(x), a, b, xi) / e_i
    return sN, sE, eps, frac


def group_luminosities(edges_Hz, T_bb: float, ndot: float) -> np.ndarray:
    """L_i in erg/s for a source emitting ndot photons/s above edges_Hz[0]
    with a blackbody spectrum (appendix on converting photon number rates)."""
    edges_eV = [H_PLANCK * e / EV if np.isfinite(e) else np.inf for e in edges_Hz]
    _, _, eps, frac = group_constants(edges_eV, T_bb)
    return eps * frac * ndot
