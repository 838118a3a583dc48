"""Drift correction on the GPU (Part III "Dealing With Particle Drifts")
against the oracle's, element by element: the GPU gradient record of a state
and the displacements in, the moved and guarded states out.

The moved state is the sum of the state and its gradient term, and can
cancel to far below either: errors are measured per state against
max(|U|, sum_a |grad U_a dx_a|) of that state (the scale of what is summed;
the GPU gradients agree with the oracle's to 1e-12 of theirs).  FP64: 1e-12;
photon totals and ledger as for the transport; guard counts exact.  FP32C:
1e-5 (FP32 gradients).  Cases: the 16^3
lattice with its strong fluxes (guards fire), every G on a ragged lattice,
a clustered Plummer set, and the whole drift-then-rebuild cycle: the moved
states on the rebuilt geometry give the oracle's next step (errors there
against the scale of each particle's neighbourhood).
"""
import numpy as np
import pytest
import torch

import oracle
import workloads
from tests.gpu_util import dev, local_err, log, unsort

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_2302_12727_amd import RT  # noqa: E402


def drift_err(got, ref, geo, U0, dx):
    dU = oracle.gradient(geo, U0)                                  # [n][G][4][3]
    term = (np.abs(dU) * np.abs(dx)[:, None, None, :]).sum(-1)     # [n][G][4]
    scale = np.maximum(np.abs(U0).max(-1), term.max(-1))
    scale = np.maximum(scale, 1e-6 * np.abs(U0[..., 0]).mean())
    return float((np.abs(got - ref).max(-1) / scale).max())


def displacements(w, scale, seed):
    return workloads.rng(seed).uniform(-scale, scale, size=(w.n, 3))


def gpu_drift(w, dx, precision="fp64"):
    rt = RT(w.n, w.groups, precision=precision)
    perm, *_ = rt.rt_build_cells(dev(w.x))
    p = perm.cpu().numpy()
    U = dev(w.U0[p]).to(rt.sdtype)
    UD = rt.rt_gradient(U)
    Q = torch.zeros(w.groups, dtype=torch.float64, device="cuda")
    counts = torch.zeros(4, dtype=torch.int64, device="cuda")
    ledger = torch.zeros(w.groups, dtype=torch.float64, device="cuda")
    out = rt.rt_drift(UD, dev(dx[p]), photon_total=Q, counts=counts, ledger=ledger)
    rt.rt_sync()
    return (unsort(out.double().cpu().numpy(), p), Q.cpu().numpy(), counts.cpu().numpy(),
            ledger.cpu().numpy())


def test_lattice16_with_guards():
    w = workloads.config(0)
    geo = oracle.build_geometry(w.x)
    dx = displacements(w, 0.3 / 16, 151)
    got, Q, counts, ledger = gpu_drift(w, dx)
    ref, rc, rl = oracle.drift(geo, w.U0, dx)
    err = drift_err(got, ref, geo, w.U0, dx)
    log(f"drift lattice16: max state err {err:.2e}; counts gpu {counts} oracle {rc}")
    assert err < 1e-12
    assert rc[2] > 0 and counts[2] == rc[2]
    assert abs(int(counts[3]) - int(rc[3])) <= 0.05 * rc[3] + 2     # ties at |F| = cE
    assert np.allclose(Q, oracle.photon_total(geo, ref), rtol=1e-12, atol=0)
    assert np.allclose(ledger, rl, rtol=1e-10, atol=1e-14)


@pytest.mark.parametrize("G", [1, 2, 5, 8])
def test_groups(G):
    w = workloads.lattice_workload(9, G, 0, 1, seed=160 + G, name="drift9")
    geo = oracle.build_geometry(w.x)
    dx = displacements(w, 0.2 / 9, 170 + G)
    got, Q, _, _ = gpu_drift(w, dx)
    ref, _, _ = oracle.drift(geo, w.U0, dx)
    assert drift_err(got, ref, geo, w.U0, dx) < 1e-12
    assert np.allclose(Q, oracle.photon_total(geo, ref), rtol=1e-12, atol=0)


def test_plummer():
    w = workloads.config(2, scale=(1 << 13) / (1 << 22))
    geo = oracle.build_geometry(w.x)
    dx = 0.2 * geo.h[:, None] * workloads.rng(181).uniform(-1, 1, size=(w.n, 3))
    got, _, _, _ = gpu_drift(w, dx)
    ref, _, _ = oracle.drift(geo, w.U0, dx)
    err = drift_err(got, ref, geo, w.U0, dx)
    log(f"drift plummer n={w.n}: max state err {err:.2e}")
    assert err < 1e-12


def test_fp32c():
    w = workloads.lattice_workload(12, 3, 0, 1, seed=191, name="drift32")
    geo = oracle.build_geometry(w.x)
    dx = displacements(w, 0.2 / 12, 192)
    got, _, _, _ = gpu_drift(w, dx, precision="fp32c")
    U32 = w.U0.astype(np.float32).astype(np.float64)
    ref, _, _ = oracle.drift(geo, U32, dx)
    err = drift_err(got, ref, geo, U32, dx)
    log(f"drift FP32C: max state err {err:.2e}")
    assert err < 1e-5


def test_drift_then_rebuild():
    w = workloads.lattice_workload(10, 2, 2, 1, seed=201, name="cycle")
    geo = oracle.build_geometry(w.x)
    dx = displacements(w, 0.15 / 10, 202)
    x1 = np.mod(w.x + dx, 1.0)
    # oracle: move the states, then one step on the geometry of the new positions
    moved, _, _ = oracle.drift(geo, w.U0, dx)
    geo1 = oracle.build_geometry(x1)
    srcs1 = oracle.build_sources(geo1, w.xs)
    ref, _ = oracle.step(geo1, srcs1, moved, w.L)
    # GPU: the same with rt_drift, rt_build_cells at x1 and one step
    got_moved = gpu_drift(w, dx)[0]
    rt = RT(w.n, w.groups)
    perm, *_ = rt.rt_build_cells(dev(x1))
    rt.rt_set_sources(dev(w.xs))
    p = perm.cpu().numpy()
    U = rt.step(dev(got_moved[p]), dev(w.L))
    rt.rt_sync()
    got = unsort(U.cpu().numpy(), p)
    # states the drift emptied take their values from their neighbours in the
    # step: errors against the neighbourhood's scale
    err = local_err(got, ref, geo1.sptr, geo1.sidx)
    log(f"drift + rebuild + step: max error {err:.2e} of the neighbourhood scale")
    assert err < 1e-12
