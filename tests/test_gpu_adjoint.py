"""Adjoint of the transport step on the GPU against the differentiable torch
reference (oracle/torch_ref.py, itself pinned to the C oracle and to finite
differences) and against finite differences of the GPU forward.

Tolerances: adjoint vs reference gradient 1e-9 relative (FP64, both exact
derivatives of the same function up to rounding); against central finite
differences 1e-6 relative (the target of the method), taking the best of a few
step sizes to stay clear of minmod and guard switches.
"""
import numpy as np
import pytest
import torch

import oracle
import workloads
from oracle.torch_ref import TorchStep
from tests.gpu_util import dev, log, unsort

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_2302_12727_amd import RT  # noqa: E402
from paper_2302_12727_amd.rollout import rollout  # noqa: E402


@pytest.fixture(scope="module")
def case():
    w = workloads.lattice_workload(10, 2, 3, 6, seed=555, name="adj")
    log(f"adjoint case lattice10 G=2 S=3 n={w.n}")
    geo = oracle.build_geometry(w.x)
    srcs = oracle.build_sources(geo, w.xs)
    ts = TorchStep(geo, srcs)
    rt = RT(w.n, w.groups)
    perm, *_ = rt.rt_build_cells(dev(w.x), dev(geo.h))
    rt.rt_set_sources(dev(w.xs))
    rt.rt_sync()
    p = perm.cpu().numpy()
    g = workloads.rng(556)
    probes = np.sort(g.choice(w.n, 96, replace=False))
    Et = g.lognormal(size=(96, w.groups))
    return w, geo, ts, rt, p, probes, Et


def rel(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


def test_single_step_vjp(case):
    w, geo, ts, rt, p, _, _ = case
    g = workloads.rng(9)
    lam_next = g.normal(size=w.U0.shape)
    U = torch.from_numpy(w.U0.copy()).requires_grad_(True)
    L = torch.from_numpy(w.L.copy()).requires_grad_(True)
    out = ts.step(U, L, geo.dt)
    gU, gL = torch.autograd.grad(out, (U, L), grad_outputs=torch.from_numpy(lam_next))
    dLdL = torch.zeros(w.L.shape, dtype=torch.float64, device="cuda")
    lam = rt.rt_adjoint(dev(w.U0[p]), dev(w.L), dev(lam_next[p]), dL_dL=dLdL)
    got = unsort(lam.cpu().numpy(), p)
    e1, e2 = rel(got, gU.numpy()), rel(dLdL.cpu().numpy(), gL.numpy())
    log(f"single-step VJP: dU rel err {e1:.2e}, dL rel err {e2:.2e}")
    assert e1 < 1e-9 and e2 < 1e-9


@pytest.mark.parametrize("n_side,groups", [(9, 1), (11, 3)])
def test_single_step_vjp_ragged(n_side, groups):
    """The adjoint's tile pair pass and its neighbour-union transposed gradient
    at 1 and 3 groups on lattices whose last tile is partial (729 and 1331
    particles), against the torch reference."""
    w = workloads.lattice_workload(n_side, groups, 2, 1, seed=700 + n_side, name="adj-ragged")
    log(f"case adjoint ragged lattice{n_side} G={groups} n={w.n}")
    geo = oracle.build_geometry(w.x)
    srcs = oracle.build_sources(geo, w.xs)
    ts = TorchStep(geo, srcs)
    rt = RT(w.n, w.groups)
    perm, *_ = rt.rt_build_cells(dev(w.x), dev(geo.h))
    rt.rt_set_sources(dev(w.xs))
    p = perm.cpu().numpy()
    g = workloads.rng(710 + n_side)
    lam_next = g.normal(size=w.U0.shape)
    U = torch.from_numpy(w.U0.copy()).requires_grad_(True)
    L = torch.from_numpy(w.L.copy()).requires_grad_(True)
    out = ts.step(U, L, geo.dt)
    gU, gL = torch.autograd.grad(out, (U, L), grad_outputs=torch.from_numpy(lam_next))
    dLdL = torch.zeros(w.L.shape, dtype=torch.float64, device="cuda")
    lam = rt.rt_adjoint(dev(w.U0[p]), dev(w.L), dev(lam_next[p]), dL_dL=dLdL)
    st = rt.rt_get_stats()
    got = unsort(lam.cpu().numpy(), p)
    e1, e2 = rel(got, gU.numpy()), rel(dLdL.cpu().numpy(), gL.numpy())
    log(f"ragged VJP lattice{n_side} G={groups}: dU rel err {e1:.2e}, dL rel err {e2:.2e}; "
        f"transposed gradient: {st['adj_union_blocks']} union blocks, "
        f"{st['adj_union_staged_blocks']} staged")
    assert st["adj_union_blocks"] + st["adj_union_staged_blocks"] == (w.n + 63) // 64
    assert e1 < 1e-9 and e2 < 1e-9


def test_vjp_with_stored_records_equals_recompute(case):
    w, geo, ts, rt, p, _, _ = case
    g = workloads.rng(10)
    lam_next = dev(g.normal(size=w.U0.shape)[p])
    U = dev(w.U0[p])
    L = dev(w.L)
    a = rt.rt_adjoint(U, L, lam_next.clone())
    U1 = U.clone()
    rt.rt_inject(U1, L)
    UD = rt.rt_gradient(U1)
    Uu = torch.empty_like(U)
    rt.rt_transport(UD, U_unguarded=Uu)
    b = rt.rt_adjoint(None, L, lam_next.clone(), UD=UD, U_unguarded=Uu)
    assert torch.equal(a, b)


def test_rollout_gradient_vs_reference(case):
    w, geo, ts, rt, p, probes, Et = case
    steps = w.steps
    U0 = torch.from_numpy(w.U0.copy()).requires_grad_(True)
    L = torch.from_numpy(w.L.copy()).requires_grad_(True)
    U = ts.run(U0, L, geo.dt, steps)
    loss = ((U[probes, :, 0] - torch.from_numpy(Et)) ** 2).sum()
    gU_ref, gL_ref = torch.autograd.grad(loss, (U0, L))
    # GPU: probes in Morton order
    inv = np.empty_like(p)
    inv[p] = np.arange(w.n)
    pr = torch.as_tensor(inv[probes], device="cuda")
    U0d = dev(w.U0[p]).requires_grad_(True)
    Ld = dev(w.L).requires_grad_(True)
    Ud = rollout(rt, Ld, U0d, steps, ckpt_every=2)
    lossd = ((Ud[pr, :, 0] - dev(Et)) ** 2).sum()
    lossd.backward()
    assert float(lossd) == pytest.approx(float(loss), rel=1e-12)
    gU = unsort(U0d.grad.cpu().numpy(), p)
    e1, e2 = rel(gU, gU_ref.numpy()), rel(Ld.grad.cpu().numpy(), gL_ref.numpy())
    log(f"{steps}-step rollout (checkpoint every 2): dU0 rel err {e1:.2e}, dL rel err {e2:.2e}")
    assert e1 < 1e-9 and e2 < 1e-9


def test_rollout_gradient_vs_finite_differences(case):
    w, geo, ts, rt, p, probes, Et = case
    steps = w.steps
    inv = np.empty_like(p)
    inv[p] = np.arange(w.n)
    pr = torch.as_tensor(inv[probes], device="cuda")
    Etd = dev(Et)
    U0d = dev(w.U0[p])

    def loss_of(L):
        with torch.no_grad():
            U = rollout(rt, L, U0d, steps, ckpt_every=3)
            return float(((U[pr, :, 0] - Etd) ** 2).sum())

    Ld = dev(w.L).requires_grad_(True)
    U = rollout(rt, Ld, U0d.clone().requires_grad_(True), steps, ckpt_every=3)
    ((U[pr, :, 0] - Etd) ** 2).sum().backward()
    gL = Ld.grad.cpu().numpy()
    worst = 0.0
    for s in range(w.L.shape[0]):
        for grp in range(w.groups):
            best = np.inf
            for r in (1e-4, 1e-5, 1e-6):
                eps = r * w.L[s, grp]
                Lp, Lm = w.L.copy(), w.L.copy()
                Lp[s, grp] += eps
                Lm[s, grp] -= eps
                fd = (loss_of(dev(Lp)) - loss_of(dev(Lm))) / (2 * eps)
                best = min(best, abs(fd - gL[s, grp]) / abs(fd))
            worst = max(worst, best)
            assert best < 1e-6, (s, grp, gL[s, grp])
    log(f"dLoss/dL vs central differences: worst rel err {worst:.2e}")


def test_dot_product_identity(case):
    """<lam, J v> = <J^T lam, v> with J v from central differences of one step."""
    w, geo, ts, rt, p, _, _ = case
    g = workloads.rng(11)
    lam = dev(g.normal(size=w.U0.shape)[p])
    v = dev(g.normal(size=w.U0.shape)[p])
    U = dev(w.U0[p])
    L = dev(w.L)
    JTlam = rt.rt_adjoint(U, L, lam.clone())
    rhs = float((JTlam * v).sum())
    best = np.inf
    for eps in (1e-5, 1e-6, 1e-7):
        Up = (U + eps * v).contiguous()
        Um = (U - eps * v).contiguous()
        Jv = (rt.step(Up, L) - rt.step(Um, L)) / (2 * eps)
        lhs = float((lam * Jv).sum())
        best = min(best, abs(lhs - rhs) / abs(rhs))
    log(f"dot-product identity rel err {best:.2e}")
    assert best < 1e-6


def test_fp32c_adjoint_against_fp64_adjoint(case):
    """Same rollout and loss in both precisions: the compensated-FP32 gradients
    against the FP64 ones (reported; bound 1e-4 normwise)."""
    w, geo, ts, rt64, p, probes, Et = case
    inv = np.empty_like(p)
    inv[p] = np.arange(w.n)
    pr = torch.as_tensor(inv[probes], device="cuda")
    rt32 = RT(w.n, w.groups, precision="fp32c")
    perm32, *_ = rt32.rt_build_cells(dev(w.x), dev(geo.h))
    rt32.rt_set_sources(dev(w.xs))
    assert np.array_equal(perm32.cpu().numpy(), p)
    grads = {}
    for name, rt, dt in (("fp64", rt64, torch.float64), ("fp32c", rt32, torch.float32)):
        U0 = dev(w.U0[p]).to(dt).requires_grad_(True)
        L = dev(w.L).requires_grad_(True)
        U = rollout(rt, L, U0, w.steps, ckpt_every=3)
        ((U[pr, :, 0].double() - dev(Et)) ** 2).sum().backward()
        grads[name] = (U0.grad.double().cpu().numpy(), L.grad.cpu().numpy())
    eU = rel(grads["fp32c"][0], grads["fp64"][0])
    eL = rel(grads["fp32c"][1], grads["fp64"][1])
    d = np.abs(grads["fp32c"][0] - grads["fp64"][0]) / np.abs(grads["fp64"][0]).max()
    q = np.quantile(d, [0.5, 0.99, 0.999])
    nbad = int((d > 1e-5).sum())
    log(f"fp32c adjoint vs fp64 adjoint: dU0 rel err max {eU:.2e} (median {q[0]:.1e}, "
        f"p99 {q[1]:.1e}, p99.9 {q[2]:.1e}, {nbad} of {d.size} entries above 1e-5), "
        f"dL rel err {eL:.2e}")
    assert eL < 1e-4
    assert q[1] < 1e-5 and eU < 1e-3
