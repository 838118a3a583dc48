"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module only draws random numbers and arranges them into arrays: it holds
none of the transport method's arithmetic.  Every generator takes an explicit
seed (NumPy PCG64) so that the oracle and the HIP path see identical inputs.

Workloads are shaped like the validation problems of the thesis (the Iliev
comparison tests of Part III: particle sets of 128^3, three photon groups split
at the HI/HeI/HeII ionisation thresholds, a few point sources; clustered
particle sets for the density-profile tests).  The suite's own initial
conditions are not reproduced; these synthetic sets stand in for them.

Units: periodic unit box [0, 1)^3, reduced speed of light c = 1.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

SEED_BASE = 12727


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def jittered_lattice(n_side: int, jitter: float, seed: int) -> np.ndarray:
    """Cubic lattice of n_side^3 points with uniform per-axis jitter.

    Point (i, j, k) sits at ((i, j, k) + 1/2 + U(-jitter, jitter)) / n_side,
    wrapped into [0, 1).  Returned in lattice order (x slowest), float64 (N, 3).
    """
    g = rng(seed)
    ax = np.arange(n_side, dtype=np.float64)
    i, j, k = np.meshgrid(ax, ax, ax, indexing="ij")
    base = np.stack([i.ravel(), j.ravel(), k.ravel()], axis=1) + 0.5
    if jitter > 0:
        base = base + g.uniform(-jitter, jitter, size=base.shape)
    x = base / n_side
    x = np.mod(x, 1.0)
    x[x >= 1.0] = 0.0
    return np.ascontiguousarray(x)


def _plummer_draw(g, n: int, scale: float, r_trunc: float, bg_frac: float) -> np.ndarray:
    """n independent draws from the Plummer + uniform-background mixture."""
    n_bg = int(g.binomial(n, bg_frac))
    n_pl = n - n_bg
    m_max = r_trunc ** 3 / (r_trunc ** 2 + scale ** 2) ** 1.5
    m = g.uniform(0.0, m_max, size=n_pl)
    m = np.maximum(m, 1e-300)
    r = scale / np.sqrt(m ** (-2.0 / 3.0) - 1.0)
    v = g.normal(size=(n_pl, 3))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    pl = 0.5 + r[:, None] * v
    bg = g.uniform(0.0, 1.0, size=(n_bg, 3))
    x = np.concatenate([pl, bg], axis=0)
    x = np.mod(x, 1.0)
    x[x >= 1.0] = 0.0
    return x


def plummer_mix(n: int, scale: float, r_trunc: float, bg_frac: float,
                seed: int, hard_core: float = 0.7) -> np.ndarray:
    """Plummer sphere (centre (1/2,1/2,1/2), scale radius `scale`, truncated at
    `r_trunc`) plus a uniform background holding `bg_frac` of the points.

    Radii use the inverse of the Plummer cumulative mass fraction
    m(r) = r^3 / (r^2 + a^2)^{3/2} with m drawn uniformly on [0, m(r_trunc)];
    directions are isotropic.

    Glass-like, not Poisson: independent draws put a few particles much closer
    together than the local spacing, and the smoothing-length equation then
    draws), which no particle set of the thesis's tests has; such particles
    make the explicit scheme unstable at any CFL number tried (down to 0.15).
    So the draws are
    thinned by a hard core (Matern type II): every candidate gets a random
    priority and is dropped if a candidate of higher priority lies within
    `hard_core` times the local mean spacing rho(x)^(-1/3) of the mixture's
    number density.  The drop rate is the same everywhere, so the density
    profile keeps its shape; enough candidates are drawn for n to survive, and
    n of the survivors are kept at random.  With the default 0.7 the fewest
    neighbours of any particle at 2^22 points is 16 and the radial profile
    matches that of plain draws bin by bin.  hard_core = 0 gives plain draws.
    Points are shuffled so that input order carries no spatial structure.
    """
    from scipy.spatial import cKDTree

    g = rng(seed)
    if hard_core <= 0:
        x = _plummer_draw(g, n, scale, r_trunc, bg_frac)
        return np.ascontiguousarray(x[g.permutation(n)])
    lam = 4.0 * np.pi / 3.0 * hard_core ** 3
    keep = (1.0 - np.exp(-lam)) / lam
    m_max = r_trunc ** 3 / (r_trunc ** 2 + scale ** 2) ** 1.5
    factor = 1.08
    while True:
        n_draw = int(n / keep * factor) + 256
        x = _plummer_draw(g, n_draw, scale, r_trunc, bg_frac)
        # number density of the mixture (n_draw points)
        rr = np.sqrt(((x - 0.5) ** 2).sum(axis=1))
        rho = bg_frac * n_draw + np.where(
            rr <= r_trunc,
            (1.0 - bg_frac) * n_draw * 3.0 / (4.0 * np.pi * scale ** 3 * m_max)
            * (1.0 + (rr / scale) ** 2) ** -2.5, 0.0)
        s = hard_core * rho ** (-1.0 / 3.0)
        prio = g.permutation(n_draw)
        tree = cKDTree(x, boxsize=1.0)
        d, nb = tree.query(x, k=9, workers=-1)
        d, nb = d[:, 1:], nb[:, 1:]
        beaten = ((d < s[:, None]) & (prio[np.minimum(nb, n_draw - 1)] < prio[:, None])).any(axis=1)
        del tree, d, nb
        survivors = np.flatnonzero(~beaten)
        if survivors.size >= n:
            break
        factor *= 1.1
    pick = g.choice(survivors, size=n, replace=False)
    return np.ascontiguousarray(x[pick[g.permutation(n)]])


def radiation_fields(n: int, groups: int, c: float, seed: int,
                     sigma: float = 1.0, fmax: float = 0.9) -> np.ndarray:
    """Initial photon state, float64 (N, G, 4) = (E, Fx, Fy, Fz) per group.

    E ~ LogNormal(0, sigma); F = u * fmax * c * E * n with n uniform on the
    unit sphere and u ~ U[0, 1], drawn independently per particle and group.
    """
    g = rng(seed)
    E = g.lognormal(mean=0.0, sigma=sigma, size=(n, groups))
    d = g.normal(size=(n, groups, 3))
    d /= np.linalg.norm(d, axis=2, keepdims=True)
    u = g.uniform(0.0, 1.0, size=(n, groups))
    F = (u * fmax * c * E)[:, :, None] * d
    U = np.empty((n, groups, 4), dtype=np.float64)
    U[:, :, 0] = E
    U[:, :, 1:] = F
    return U


def sources_at_particles(x: np.ndarray, n_src: int, groups: int, seed: int,
                         lum_lo: float = 1e-2, lum_hi: float = 1.0):
    """`n_src` point sources placed on distinct random particles, luminosities
    log-uniform on [lum_lo, lum_hi] per source and group."""
    g = rng(seed)
    idx = g.choice(x.shape[0], size=n_src, replace=False)
    xs = np.ascontiguousarray(x[idx].copy())
    L = np.exp(g.uniform(math.log(lum_lo), math.log(lum_hi), size=(n_src, groups)))
    return xs, np.ascontiguousarray(L)


@dataclasses.dataclass
class Workload:
    name: str
    x: np.ndarray                 # (N, 3) float64 positions in [0,1)
    U0: np.ndarray                # (N, G, 4) float64 initial photon state
    xs: np.ndarray                # (S, 3) source positions (S may be 0)
    L: np.ndarray                 # (S, G) luminosities
    steps: int
    groups: int
    c_red: float = 1.0
    cfl: float = 0.9
    eta: float = 1.2348
    eta_star: float = 1.2348
    probes: Optional[np.ndarray] = None   # probe particle indices (input order)
    L_target: Optional[np.ndarray] = None  # luminosities of the target run
    ckpt_every: int = 0

    @property
    def n(self) -> int:
        return self.x.shape[0]


def lattice_workload(n_side: int, groups: int, n_src: int, steps: int, seed: int,
                     name: str = "lattice", jitter: float = 0.1) -> Workload:
    x = jittered_lattice(n_side, jitter, seed)
    U0 = radiation_fields(x.shape[0], groups, 1.0, seed + 1000)
    if n_src > 0:
        xs, L = sources_at_particles(x, n_src, groups, seed + 2000)
    else:
        xs, L = np.zeros((0, 3)), np.zeros((0, groups))
    return Workload(name, x, U0, xs, L, steps, groups)


def plummer_workload(n: int, groups: int, steps: int, seed: int, n_src: int = 1,
                     name: str = "plummer", central_source: bool = True) -> Workload:
    x = plummer_mix(n, 0.05, 0.5, 0.1, seed)
    U0 = radiation_fields(n, groups, 1.0, seed + 1000)
    if central_source:
        xs = np.full((1, 3), 0.5)
        L = np.ones((1, groups))
    elif n_src > 0:
        xs, L = sources_at_particles(x, n_src, groups, seed + 2000)
    else:
        xs, L = np.zeros((0, 3)), np.zeros((0, groups))
    return Workload(name, x, U0, xs, L, steps, groups)


def config(index: int, scale: float = 1.0) -> Workload:
    """The five benchmark configurations (index 0..4).

    `scale` < 1 shrinks the particle count (keeping the recipe) for tests that
    must finish quickly; scale = 1 is the full size.
    """
    seed = SEED_BASE + index
    if index == 0:
        # 16^3 jittered lattice, one group, no sources, 10 steps (FP64).
        n_side = max(6, int(round(16 * scale ** (1 / 3))))
        return lattice_workload(n_side, 1, 0, 10, seed, "lattice16_g1")
    if index == 1:
        # 128^3 jittered lattice, three groups, 16 sources, 100 steps (FP64).
        n_side = max(8, int(round(128 * scale ** (1 / 3))))
        return lattice_workload(n_side, 3, 16, 100, seed, f"lattice{n_side}_g3_s16")
    if index == 2:
        # 2^22 Plummer + 10% background, three groups, central source, 100 steps.
        n = max(4096, int(round((1 << 22) * scale)))
        return plummer_workload(n, 3, 100, seed, name=f"plummer{n}_g3_s1")
    if index == 3:
        # 2^20 lattice, three groups, 64 sources, 20 steps, adjoint.
        n_side = max(8, int(round(128 * scale ** (1 / 3))))
        w = lattice_workload(n_side, 3, 64, 20, seed, f"lattice{n_side}_g3_s64_adj")
        g = rng(seed + 3000)
        n_probe = min(4096, w.n)
        w.probes = np.sort(g.choice(w.n, size=n_probe, replace=False))
        w.L_target = w.L * np.exp(0.1 * g.normal(size=w.L.shape))
        w.ckpt_every = 5
        return w
    if index == 4:
        # 2^24 Plummer + background, four groups, 256 sources, 50 steps, adjoint.
        n = max(4096, int(round((1 << 24) * scale)))
        w = plummer_workload(n, 4, 50, seed, n_src=256, name=f"plummer{n}_g4_s256_adj",
                             central_source=False)
        g = rng(seed + 3000)
        n_probe = min(4096, w.n)
        w.probes = np.sort(g.choice(w.n, size=n_probe, replace=False))
        w.L_target = w.L * np.exp(0.1 * g.normal(size=w.L.shape))
        w.ckpt_every = 10
        return w
    raise ValueError(f"unknown config index {index}")


def perfect_lattice(n_side: int) -> np.ndarray:
    """Unjittered cubic lattice ((i,j,k)+1/2)/n_side."""
    return jittered_lattice(n_side, 0.0, 0)
