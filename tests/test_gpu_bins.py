"""Individual time steps on the GPU against the oracle (Part II "Individual
time steps", Part III eq:transport-update-explicit with min{dt_k, dt_l}, the
factor-4 limiter).

- time bins equal the oracle's (exact);
- max_bin = 0 reproduces the global step (1e-12 per state);
- two full cycles of a clustered set with sources: states and pending flux
  sums against the oracle (1e-12 per state; sums against the state scale);
- the photon budget including the pending sums closes every tick (1e-12);
- the Ivanova surfaces (GLF and HLL): two cycles and a mid-cycle state with
  pending sums against the oracle's binned scheme with those surfaces;
- FP32C contexts (GLF, HLL, Ivanova): two cycles and a mid-cycle state against
  the FP64 oracle at the FP32C bar, and the budget with pending sums (1e-6).
"""
import numpy as np
import pytest
import torch

import oracle
import workloads
from tests.gpu_util import dev, local_err, log, state_err, unsort

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_2302_12727_amd import RT  # noqa: E402

MAX_BIN = 6


@pytest.fixture(scope="module")
def case():
    w = workloads.config(2, scale=(1 << 13) / (1 << 22))     # 8192 Plummer + background
    log(f"time-bin case plummer n={w.n} G={w.groups}")
    geo = oracle.build_geometry(w.x)
    srcs = oracle.build_sources(geo, w.xs)
    rt = RT(w.n, w.groups, cfl=w.cfl, c_red=w.c_red)
    perm, *_ = rt.rt_build_cells(dev(w.x), dev(geo.h))
    rt.rt_set_sources(dev(w.xs))
    rt.rt_sync()
    return w, geo, srcs, rt, perm.cpu().numpy()


def gpu_ticks(rt, w, p, ticks, U0=None):
    U = dev((w.U0 if U0 is None else U0)[p])
    L = dev(w.L)
    UD = rt.rt_gradient(U)
    acc = torch.zeros_like(U)
    Q = torch.zeros(w.groups, dtype=torch.float64, device="cuda")
    ledger = torch.zeros(w.groups, dtype=torch.float64, device="cuda")
    for t in range(ticks):
        rt.rt_tick(U, L, t, UD, acc, photon_total=Q, ledger=ledger)
    rt.rt_sync()
    return U, acc, Q, ledger


def test_bins_equal_oracle(case):
    w, geo, srcs, rt, p = case
    bins, cycle = rt.rt_time_bins(MAX_BIN)
    got = unsort(bins.cpu().numpy(), p)
    ref = oracle.time_bins(geo, MAX_BIN)
    log(f"bins: counts {np.bincount(ref)}, cycle {cycle} ticks")
    assert np.array_equal(got, ref)
    assert cycle == 1 << int(ref.max())


def test_bin_zero_is_the_global_step(case):
    w, geo, srcs, rt, p = case
    rt.rt_time_bins(0)
    U, acc, _, _ = gpu_ticks(rt, w, p, 3)
    ref, _ = oracle.run(geo, srcs, w.U0, w.L, 3)
    err = state_err(unsort(U.cpu().numpy(), p), ref)
    log(f"max_bin 0, 3 ticks vs the global oracle step: {err:.2e}")
    assert err < 1e-12
    assert not acc.any()


def test_two_cycles_against_oracle(case):
    w, geo, srcs, rt, p = case
    bins, cycle = rt.rt_time_bins(MAX_BIN)
    ticks = 2 * cycle
    U, acc, Q, ledger = gpu_ticks(rt, w, p, ticks)
    ref, info = oracle.run_binned(geo, srcs, w.U0, w.L, ticks, oracle.time_bins(geo, MAX_BIN))
    got = unsort(U.cpu().numpy(), p)
    err = state_err(got, ref)
    log(f"{ticks} ticks ({cycle}-tick cycles, bins 0..{int(bins.max())}): max state err {err:.2e}")
    assert err < 1e-12
    assert not acc.any()                        # every particle has just ended a step
    assert np.allclose(ledger.cpu().numpy(), info["ledger"], rtol=1e-10, atol=1e-14)
    Qo = oracle.photon_total(geo, ref)
    assert np.allclose(Q.cpu().numpy(), Qo, rtol=1e-12, atol=0)


def test_mid_cycle_pending_sums(case):
    w, geo, srcs, rt, p = case
    bins, cycle = rt.rt_time_bins(MAX_BIN)
    ticks = cycle + cycle // 2 + 1              # mid-cycle: pending sums exist
    U, acc, _, _ = gpu_ticks(rt, w, p, ticks)
    ref, info = oracle.run_binned(geo, srcs, w.U0, w.L, ticks, oracle.time_bins(geo, MAX_BIN))
    assert state_err(unsort(U.cpu().numpy(), p), ref) < 1e-12
    acc_got = unsort(acc.cpu().numpy(), p)
    scale = np.abs(ref).max() * geo.V.max()
    err = float(np.abs(acc_got - info["acc"]).max() / scale)
    log(f"pending flux sums after {ticks} ticks: max err {err:.2e} of V E")
    assert info["acc"].any() and err < 1e-12


def test_budget_with_pending_sums_every_tick(case):
    w, geo, srcs, rt, p = case
    bins, cycle = rt.rt_time_bins(3)
    U = dev(w.U0[p])
    L = dev(w.L)
    UD = rt.rt_gradient(U)
    acc = torch.zeros_like(U)
    Q = torch.zeros(w.groups, dtype=torch.float64, device="cuda")
    ledger = torch.zeros(w.groups, dtype=torch.float64, device="cuda")
    Q0 = rt.rt_photon_total(U).cpu().numpy()
    dt = float(rt.dt.item())
    worst = 0.0
    for t in range(2 * cycle):
        rt.rt_tick(U, L, t, UD, acc, photon_total=Q, ledger=ledger)
        pending = acc[:, :, 0].sum(dim=0).cpu().numpy()
        lhs = Q.cpu().numpy() - pending
        rhs = Q0 + (t + 1) * dt * w.L.sum(axis=0) + ledger.cpu().numpy()
        worst = max(worst, float(np.abs(lhs / rhs - 1).max()))
    log(f"budget with pending sums over {2 * cycle} ticks: worst {worst:.2e}")
    assert worst < 1e-12


@pytest.mark.parametrize("solver", ["glf", "hll"])
def test_ivanova_against_oracle(case, solver):
    """Individual time bins with the Ivanova surfaces (Part II eq:IvanovaAij):
    two cycles, then a mid-cycle state with pending sums."""
    w, geo, srcs, rt, p = case
    tab = oracle.hll_table() if solver == "hll" else None
    rt.rt_set_surfaces("ivanova")
    rt.rt_set_riemann(solver)
    try:
        bins, cycle = rt.rt_time_bins(MAX_BIN)
        ob = oracle.time_bins(geo, MAX_BIN)
        for ticks in (2 * cycle, cycle + cycle // 2 + 1):
            U, acc, Q, _ = gpu_ticks(rt, w, p, ticks)
            ref, info = oracle.run_binned(geo, srcs, w.U0, w.L, ticks, ob, hll=tab, ivanova=True)
            err = state_err(unsort(U.cpu().numpy(), p), ref)
            scale = np.abs(ref).max() * geo.V.max()
            aerr = float(np.abs(unsort(acc.cpu().numpy(), p) - info["acc"]).max() / scale)
            log(f"Ivanova {solver} {ticks} ticks: max state err {err:.2e}, pending sums {aerr:.2e}")
            assert err < 1e-12 and aerr < 1e-12
            assert np.allclose(Q.cpu().numpy(), oracle.photon_total(geo, ref), rtol=1e-12, atol=0)
        hop, _ = oracle.run_binned(geo, srcs, w.U0, w.L, ticks, ob, hll=tab)
        assert state_err(unsort(U.cpu().numpy(), p), hop) > 1e-6
    finally:
        rt.rt_set_surfaces("hopkins")
        rt.rt_set_riemann("glf")


@pytest.fixture(scope="module")
def case32(case):
    w, geo, srcs, _, p = case
    rt = RT(w.n, w.groups, precision="fp32c", cfl=w.cfl, c_red=w.c_red)
    perm, *_ = rt.rt_build_cells(dev(w.x), dev(geo.h))
    rt.rt_set_sources(dev(w.xs))
    rt.rt_sync()
    assert np.array_equal(perm.cpu().numpy(), p)
    return rt


def gpu_ticks32(rt, w, p, ticks):
    U = dev(w.U0[p]).float()
    L = dev(w.L)
    UD = rt.rt_gradient(U)
    acc = torch.zeros(U.shape, dtype=torch.float64, device="cuda")
    Q = torch.zeros(w.groups, dtype=torch.float64, device="cuda")
    ledger = torch.zeros(w.groups, dtype=torch.float64, device="cuda")
    for t in range(ticks):
        rt.rt_tick(U, L, t, UD, acc, photon_total=Q, ledger=ledger)
    rt.rt_sync()
    return U, acc, Q, ledger


@pytest.mark.parametrize("variant", ["glf", "hll", "ivanova"])
def test_fp32c_against_oracle(case, case32, variant):
    """Individual time bins in an FP32C context against the FP64 oracle's binned
    scheme: two cycles and a mid-cycle state, at the FP32C bar (1e-5 of each
    neighbourhood's scale; pending sums against V times the state scale)."""
    w, geo, srcs, _, p = case
    rt = case32
    tab = oracle.hll_table() if variant == "hll" else None
    rt.rt_set_riemann("hll" if variant == "hll" else "glf")
    rt.rt_set_surfaces("ivanova" if variant == "ivanova" else "hopkins")
    try:
        bins, cycle = rt.rt_time_bins(MAX_BIN)
        ob = oracle.time_bins(geo, MAX_BIN)
        assert np.array_equal(unsort(bins.cpu().numpy(), p), ob)
        for ticks in (2 * cycle, cycle + cycle // 2 + 1):
            U, acc, Q, _ = gpu_ticks32(rt, w, p, ticks)
            ref, info = oracle.run_binned(geo, srcs, w.U0, w.L, ticks, ob, hll=tab,
                                          ivanova=variant == "ivanova")
            err = local_err(unsort(U.double().cpu().numpy(), p), ref, geo.sptr, geo.sidx)
            scale = np.abs(ref).max() * geo.V.max()
            aerr = float(np.abs(unsort(acc.cpu().numpy(), p) - info["acc"]).max() / scale)
            log(f"FP32C {variant} {ticks} ticks: max err {err:.2e} of the neighbourhood scale, "
                f"pending sums {aerr:.2e}")
            assert err < 1e-5 and aerr < 1e-5
            assert np.allclose(Q.cpu().numpy(), oracle.photon_total(geo, ref), rtol=1e-6, atol=0)
    finally:
        rt.rt_set_riemann("glf")
        rt.rt_set_surfaces("hopkins")


def test_fp32c_budget_with_pending_sums_every_tick(case, case32):
    w, geo, srcs, _, p = case
    rt = case32
    bins, cycle = rt.rt_time_bins(3)
    U = dev(w.U0[p]).float()
    L = dev(w.L)
    UD = rt.rt_gradient(U)
    acc = torch.zeros(U.shape, dtype=torch.float64, device="cuda")
    Q = torch.zeros(w.groups, dtype=torch.float64, device="cuda")
    ledger = torch.zeros(w.groups, dtype=torch.float64, device="cuda")
    Q0 = rt.rt_photon_total(U).cpu().numpy()
    dt = float(rt.dt.item())
    worst = 0.0
    for t in range(2 * cycle):
        rt.rt_tick(U, L, t, UD, acc, photon_total=Q, ledger=ledger)
        lhs = Q.cpu().numpy() - acc[:, :, 0].sum(dim=0).cpu().numpy()
        rhs = Q0 + (t + 1) * dt * w.L.sum(axis=0) + ledger.cpu().numpy()
        worst = max(worst, float(np.abs(lhs / rhs - 1).max()))
    log(f"FP32C budget with pending sums over {2 * cycle} ticks: worst {worst:.2e}")
    assert worst < 1e-6
