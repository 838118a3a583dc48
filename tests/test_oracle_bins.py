"""Pins of the oracle's individual-time-step scheme (Part II "Individual time
steps", eq:meshless-explicit-individual-timesteps; Part III
eq:transport-update-explicit with min{dt_k, dt_l}; the factor-4 limiter of
Part III "Dynamic Sub-Cycling").

- bins: within each particle's own CFL step, interacting pairs at most 2 bins
  apart, and equal to the greatest such assignment computed independently here
  (min over neighbours j of the CFL bin of j plus 2 per hop);
- all bins 0 is the global-step scheme; all bins 1 for two ticks is one global
  step of 2 dt_min (pins the time integration with min{dt_k, dt_l}); both to
  the FP64 parity bar of 1e-12 per state (the binned scheme multiplies each
  pair exchange by its dt before summing, the global one the sum by dt/V);
- photon budget at every tick including the pending flux sums:
  sum_k (V_k E_k - acc_k,E) = Q0 + injected + ledger; at a tick where every
  particle ends a step the sums are empty.
"""
import numpy as np
import pytest

import oracle
import workloads


@pytest.fixture(scope="module")
def clustered(orc):
    w = workloads.config(2, scale=(1 << 12) / (1 << 22))      # 4096 Plummer + background
    geo = oracle.build_geometry(w.x)
    srcs = oracle.build_sources(geo, w.xs)
    return w, geo, srcs


def state_err(got, ref):
    """Largest per-state error relative to max(E, |F|/c) of that state, the
    scale floored at 1e-6 of the mean energy (states a guard emptied are 0)."""
    scale = np.maximum(np.abs(ref).max(axis=-1), 1e-6 * np.abs(ref[..., 0]).mean())
    return float((np.abs(got - ref).max(axis=-1) / scale).max())


def cfl_bins(geo, nmax):
    dx = np.cbrt(geo.V / (4.0 * np.pi / 3.0))
    tau = geo.cfl * dx / geo.c
    b = np.zeros(geo.n, dtype=np.int64)
    for n in range(1, nmax + 1):
        b[geo.dt * 2.0 ** n <= tau] = n
    return b


def test_bins_properties_and_greatest(clustered):
    w, geo, _ = clustered
    nmax = 6
    b = oracle.time_bins(geo, nmax).astype(np.int64)
    own = cfl_bins(geo, nmax)
    assert (b <= own).all() and b.min() == 0
    rows = np.repeat(np.arange(geo.n), np.diff(geo.sptr))
    assert (np.abs(b[rows] - b[geo.sidx]) <= 2).all()
    # greatest assignment: relax b_i <- min(b_i, b_j + 2) from the CFL bins by
    # whole-array sweeps (Bellman-Ford on the neighbour graph)
    ref = own.copy()
    while True:
        cand = ref.copy()
        np.minimum.at(cand, rows, ref[geo.sidx] + 2)
        if np.array_equal(cand, ref):
            break
        ref = cand
    assert np.array_equal(b, ref)
    assert len(np.unique(b)) >= 3          # the clustered set spreads over several bins


def test_bins_zero_is_the_global_step(clustered):
    w, geo, srcs = clustered
    ref, _ = oracle.run(geo, srcs, w.U0, w.L, 3)
    got, info = oracle.run_binned(geo, srcs, w.U0, w.L, 3, np.zeros(geo.n, np.int32))
    assert state_err(got, ref) < 1e-12
    assert not info["acc"].any()


def test_bins_one_is_a_global_step_of_twice_dt(clustered):
    w, geo, srcs = clustered
    ref, _ = oracle.step(geo, srcs, w.U0, w.L, dt=2.0 * geo.dt)
    got, info = oracle.run_binned(geo, srcs, w.U0, w.L, 2, np.ones(geo.n, np.int32))
    assert state_err(got, ref) < 1e-12


def test_budget_with_pending_sums_every_tick(clustered):
    w, geo, srcs = clustered
    bins = oracle.time_bins(geo, 3)
    top = int(bins.max())
    U = w.U0.copy()
    Q0 = oracle.photon_total(geo, U)
    dU, acc = None, None
    ledger = np.zeros(w.groups)
    for t in range(2 << top):
        U, info = oracle.run_binned(geo, srcs, U, w.L, 1, bins, t0=t, dU=dU, acc=acc)
        dU, acc = info["dU"], info["acc"]
        ledger += info["ledger"]
        pending = acc[:, :, 0].sum(axis=0)
        injected = (t + 1) * geo.dt * w.L.sum(axis=0)
        lhs = oracle.photon_total(geo, U) - pending
        rhs = Q0 + injected + ledger
        assert np.abs(lhs / rhs - 1).max() < 1e-12, t
        if (t + 1) % (1 << top) == 0:
            assert not acc.any(), t


# ---------------------------------------------------------------------------
# The same reductions with the Ivanova surfaces (Part II eq:IvanovaAij), and
# the budget over a cycle of several bins (the surfaces are antisymmetric,
# so the pending sums still close it).
def test_ivanova_bins_zero_and_one(clustered):
    w, geo, srcs = clustered
    ref, _ = oracle.run(geo, srcs, w.U0, w.L, 3, ivanova=True)
    got, info = oracle.run_binned(geo, srcs, w.U0, w.L, 3, np.zeros(geo.n, np.int32),
                                  ivanova=True)
    assert state_err(got, ref) < 1e-12
    assert not info["acc"].any()
    ref2, _ = oracle.step(geo, srcs, w.U0, w.L, dt=2.0 * geo.dt, ivanova=True)
    got2, _ = oracle.run_binned(geo, srcs, w.U0, w.L, 2, np.ones(geo.n, np.int32), ivanova=True)
    assert state_err(got2, ref2) < 1e-12
    hop, _ = oracle.run_binned(geo, srcs, w.U0, w.L, 3, np.zeros(geo.n, np.int32))
    assert state_err(got, hop) > 1e-6


def test_ivanova_budget_with_pending_sums(clustered):
    w, geo, srcs = clustered
    bins = oracle.time_bins(geo, 2)
    top = int(bins.max())
    U = w.U0.copy()
    Q0 = oracle.photon_total(geo, U)
    dU, acc = None, None
    ledger = np.zeros(w.groups)
    for t in range(1 << top):
        U, info = oracle.run_binned(geo, srcs, U, w.L, 1, bins, t0=t, dU=dU, acc=acc,
                                    ivanova=True)
        dU, acc = info["dU"], info["acc"]
        ledger += info["ledger"]
        lhs = oracle.photon_total(geo, U) - acc[:, :, 0].sum(axis=0)
        rhs = Q0 + (t + 1) * geo.dt * w.L.sum(axis=0) + ledger
        assert np.abs(lhs / rhs - 1).max() < 1e-12, t
    assert not acc.any()
