"""The HLL solver on the GPU (Part III eq:riemann-HLL) against the oracle's HLL
step, element by element on the same seeded inputs.

The oracle uses its own eigenvalue table (numpy eigenvalues of a complex-step
Jacobian), the library its own (closed-form quadratic); the tables agree to
about 1e-14, so the states agree to the FP64 bar of 1e-12 per state, as for
GLF.  Cases: the 16^3 lattice (strong fluxes, guards firing), 3 groups with
sources (one group per wave), ragged sizes, a clustered Plummer set, photon
conservation without guards, the switch back to GLF, individual time bins
(mid-cycle states and pending flux sums against the oracle's binned HLL
scheme), the compensated-FP32 kernel (1e-5 of each neighbourhood's scale, the
FP32C bar), and the refusals.
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

from paper_2302_12727_amd import RT, RTError  # noqa: E402

TOL = 1e-12


@pytest.fixture(scope="module")
def tab():
    return oracle.hll_table()


def gpu_case(w, cfl=0.9, solver="hll"):
    rt = RT(w.n, w.groups, cfl=cfl)
    perm, *_ = rt.rt_build_cells(dev(w.x))
    if w.xs.shape[0]:
        rt.rt_set_sources(dev(w.xs))
    rt.rt_set_riemann(solver)
    rt.rt_sync()
    return rt, perm.cpu().numpy()


def run_gpu(rt, p, w, steps, U0=None):
    U = dev((w.U0 if U0 is None else U0)[p])
    L = dev(w.L) if w.xs.shape[0] else None
    counts = torch.zeros(4, dtype=torch.int64, device="cuda")
    ledger = torch.zeros(w.groups, dtype=torch.float64, device="cuda")
    Q = torch.zeros(w.groups, dtype=torch.float64, device="cuda")
    for _ in range(steps):
        U = rt.step(U, L, photon_total=Q, counts=counts, ledger=ledger)
    rt.rt_sync()
    return unsort(U.cpu().numpy(), p), Q.cpu().numpy(), counts.cpu().numpy(), ledger.cpu().numpy()


def test_c1_ten_steps(tab):
    w = workloads.config(0)
    log(f"HLL case C1 lattice16 n={w.n}")
    geo = oracle.build_geometry(w.x)
    rt, p = gpu_case(w)
    ref, info = oracle.run(geo, None, w.U0, None, w.steps, hll=tab)
    got, Q, counts, ledger = run_gpu(rt, p, w, w.steps)
    err = state_err(got, ref)
    log(f"HLL C1 10 steps: max state err {err:.3e}; counts gpu {counts} oracle {info['counts']}")
    assert err < TOL
    assert np.allclose(Q, oracle.photon_total(geo, ref), rtol=1e-12, atol=0)
    assert np.allclose(ledger, info["ledger"], rtol=1e-10, atol=1e-14)
    assert counts[0] == info["counts"][0] and counts[2] == info["counts"][2]
    glf, _ = oracle.run(geo, None, w.U0, None, w.steps)
    assert state_err(got, glf) > 1e-6          # a different solver from GLF


def test_groups_with_sources(tab):
    w = workloads.config(1, scale=(20 ** 3) / (128 ** 3))     # 20^3, G=3, 16 sources
    log(f"HLL case lattice20 G=3 S=16 n={w.n}")
    geo = oracle.build_geometry(w.x)
    srcs = oracle.build_sources(geo, w.xs)
    rt, p = gpu_case(w)
    ref, _ = oracle.run(geo, srcs, w.U0, w.L, 3, hll=tab)
    got, Q, _, _ = run_gpu(rt, p, w, 3)
    err = state_err(got, ref)
    log(f"HLL lattice20 3 steps: max state err {err:.3e}")
    assert err < TOL
    assert np.allclose(Q, oracle.photon_total(geo, ref), rtol=1e-12)


@pytest.mark.parametrize("n_side,groups", [(7, 2), (9, 1), (11, 4), (9, 5)])
def test_ragged_sizes(tab, n_side, groups):
    w = workloads.lattice_workload(n_side, groups, 2, 3, seed=930 + n_side, name="ragged")
    log(f"HLL case ragged lattice{n_side} G={groups} n={w.n}")
    geo = oracle.build_geometry(w.x)
    srcs = oracle.build_sources(geo, w.xs)
    rt, p = gpu_case(w)
    ref, _ = oracle.run(geo, srcs, w.U0, w.L, 3, hll=tab)
    got = run_gpu(rt, p, w, 3)[0]
    assert state_err(got, ref) < TOL


def test_plummer(tab):
    w = workloads.config(2, scale=(1 << 13) / (1 << 22))     # 8192 Plummer + background
    log(f"HLL case plummer n={w.n}")
    geo = oracle.build_geometry(w.x)
    srcs = oracle.build_sources(geo, w.xs)
    rt, p = gpu_case(w)
    ref, _ = oracle.run(geo, srcs, w.U0, w.L, 2, hll=tab)
    got = run_gpu(rt, p, w, 2)[0]
    err = state_err(got, ref)
    log(f"HLL plummer 2 steps: max state err {err:.3e}")
    assert err < TOL


def test_conservation_without_guards():
    x = workloads.jittered_lattice(16, 0.1, 5)
    g = workloads.rng(6)
    E = 1.0 + 0.3 * np.sin(2 * np.pi * x[:, 0]) * np.cos(2 * np.pi * x[:, 1])
    U0 = np.zeros((x.shape[0], 1, 4))
    U0[:, 0, 0] = E
    U0[:, 0, 1:] = 0.05 * E[:, None] * g.normal(size=(x.shape[0], 3))
    w = workloads.Workload("smooth", x, U0, np.zeros((0, 3)), np.zeros((0, 1)), 5, 1)
    rt, p = gpu_case(w, cfl=0.3)
    Q0 = rt.rt_photon_total(dev(U0[p])).item()
    _, Q, counts, _ = run_gpu(rt, p, w, 5)
    assert counts.sum() == 0
    assert abs(Q[0] - Q0) <= 1e-13 * Q0


def test_switch_back_to_glf():
    w = workloads.lattice_workload(9, 2, 2, 2, seed=941, name="switch")
    geo = oracle.build_geometry(w.x)
    srcs = oracle.build_sources(geo, w.xs)
    rt, p = gpu_case(w)
    run_gpu(rt, p, w, 1)
    rt.rt_set_riemann("glf")
    got = run_gpu(rt, p, w, 2)[0]
    ref, _ = oracle.run(geo, srcs, w.U0, w.L, 2)
    assert state_err(got, ref) < TOL


def test_refusals():
    """A solver code that does not exist.  (The FP64 adjoint takes HLL, the
    FP32C one refuses it: tests/test_gpu_adjoint_hll.py.)"""
    w = workloads.lattice_workload(7, 1, 0, 1, seed=950, name="refuse")
    rt, p = gpu_case(w)
    with pytest.raises(RTError, match="RT_EINVAL"):
        rt._check(rt.L.rt_set_riemann(rt.ctx, 7))


@pytest.mark.parametrize("case", ["lattice16", "plummer"])
def test_fp32c(tab, case):
    """The compensated-FP32 kernel with HLL against the FP64 oracle's HLL steps,
    at the FP32C bar (1e-5 of each neighbourhood's scale)."""
    if case == "lattice16":
        w, steps = workloads.config(0), 10
    else:
        w, steps = workloads.config(2, scale=(1 << 13) / (1 << 22)), 2
    geo = oracle.build_geometry(w.x)
    srcs = oracle.build_sources(geo, w.xs) if w.xs.shape[0] else None
    rt = RT(w.n, w.groups, precision="fp32c")
    perm, *_ = rt.rt_build_cells(dev(w.x))
    if w.xs.shape[0]:
        rt.rt_set_sources(dev(w.xs))
    rt.rt_set_riemann("hll")
    p = perm.cpu().numpy()
    U = dev(w.U0[p]).float()
    L = dev(w.L) if w.xs.shape[0] else None
    for _ in range(steps):
        U = rt.step(U, L)
    rt.rt_sync()
    got = unsort(U.double().cpu().numpy(), p)
    ref, _ = oracle.run(geo, srcs, w.U0, w.L if w.xs.shape[0] else None, steps, hll=tab)
    err = local_err(got, ref, geo.sptr, geo.sidx)
    log(f"HLL FP32C {case} {steps} steps: max err {err:.2e} of the neighbourhood scale")
    assert err < 1e-5


def test_time_bins_with_hll(tab):
    w = workloads.config(2, scale=(1 << 13) / (1 << 22))     # 8192 Plummer + background
    geo = oracle.build_geometry(w.x)
    srcs = oracle.build_sources(geo, w.xs)
    rt, p = gpu_case(w)
    bins, cycle = rt.rt_time_bins(6)
    ticks = cycle + cycle // 2 + 1                            # mid-cycle: pending sums exist
    U = dev(w.U0[p])
    L = dev(w.L)
    UD = rt.rt_gradient(U)
    acc = torch.zeros_like(U)
    for t in range(ticks):
        rt.rt_tick(U, L, t, UD, acc)
    rt.rt_sync()
    ref, info = oracle.run_binned(geo, srcs, w.U0, w.L, ticks, oracle.time_bins(geo, 6), hll=tab)
    err = state_err(unsort(U.cpu().numpy(), p), ref)
    acc_err = float(np.abs(unsort(acc.cpu().numpy(), p) - info["acc"]).max()
                    / (np.abs(ref).max() * geo.V.max()))
    log(f"HLL time bins, {ticks} ticks: max state err {err:.2e}, pending sums {acc_err:.2e}")
    assert err < 1e-12
    assert info["acc"].any() and acc_err < 1e-12
