"""Pins of the differentiable torch reference (oracle/torch_ref.py): its
forward equals the C oracle's, and its autograd gradients equal central finite
differences of the C oracle.  (The thesis has no adjoint; these pins are the
mathematics: forward agreement and the definition of the derivative.)"""
import numpy as np
import pytest
import torch

import oracle
import workloads
from oracle.torch_ref import TorchStep


@pytest.fixture(scope="module")
def small():
    w = workloads.lattice_workload(10, 2, 3, 3, seed=321, name="adj-small")
    geo = oracle.build_geometry(w.x)
    srcs = oracle.build_sources(geo, w.xs)
    ts = TorchStep(geo, srcs)
    g = workloads.rng(322)
    probes = np.sort(g.choice(w.n, 64, replace=False))
    Et = g.lognormal(size=(64, w.groups))
    return w, geo, srcs, ts, probes, Et


def loss_np(geo, srcs, U0, L, steps, probes, Et):
    U, _ = oracle.run(geo, srcs, U0, L, steps)
    return float(((U[probes, :, 0] - Et) ** 2).sum())


def test_forward_matches_oracle(small):
    w, geo, srcs, ts, _, _ = small
    ref, _ = oracle.run(geo, srcs, w.U0, w.L, 3)
    got = ts.run(torch.from_numpy(w.U0), torch.from_numpy(w.L), geo.dt, 3).numpy()
    scale = np.abs(ref).max(axis=-1, keepdims=True)
    assert (np.abs(got - ref) / scale).max() < 1e-12


def fd_matches(f, x0, value, scale, rel=1e-6, steps=(1e-4, 1e-5, 1e-6)):
    """Central differences of f at x0 with steps r * scale for several r: some
    step must reproduce `value` (a step may straddle a minmod or guard switch,
    or drown in rounding; then another is taken)."""
    fds = []
    for r in steps:
        eps = r * scale
        fd = (f(x0 + eps) - f(x0 - eps)) / (2 * eps)
        fds.append(fd)
        if abs(fd - value) <= rel * abs(fd) + 1e-10:
            return True, fds
    return False, fds


def test_autograd_matches_finite_differences(small):
    w, geo, srcs, ts, probes, Et = small
    U0 = torch.from_numpy(w.U0.copy()).requires_grad_(True)
    L = torch.from_numpy(w.L.copy()).requires_grad_(True)
    U = ts.run(U0, L, geo.dt, w.steps)
    loss = ((U[probes, :, 0] - torch.from_numpy(Et)) ** 2).sum()
    gL, gU = torch.autograd.grad(loss, (L, U0))
    gL, gU = gL.numpy(), gU.numpy()
    for s in range(w.L.shape[0]):
        for grp in range(w.groups):
            def f(v):
                Lx = w.L.copy()
                Lx[s, grp] = v
                return loss_np(geo, srcs, w.U0, Lx, w.steps, probes, Et)
            ok, fds = fd_matches(f, w.L[s, grp], gL[s, grp], w.L[s, grp])
            assert ok, (s, grp, gL[s, grp], fds)
    g = workloads.rng(7)
    for _ in range(12):
        i = int(g.choice(probes))
        grp, m = int(g.integers(w.groups)), int(g.integers(4))

        def f(v):
            Ux = w.U0.copy()
            Ux[i, grp, m] = v
            return loss_np(geo, srcs, Ux, w.L, w.steps, probes, Et)
        ok, fds = fd_matches(f, w.U0[i, grp, m], gU[i, grp, m], np.abs(w.U0[i, grp]).max())
        assert ok, (i, grp, m, gU[i, grp, m], fds)


# ---------------------------------------------------------------------------
# The same two pins with the HLL solver (Part III eq:riemann-HLL): forward
# against the C oracle's HLL transport, autograd against its central
# differences.
@pytest.fixture(scope="module")
def small_hll():
    w = workloads.lattice_workload(10, 2, 3, 3, seed=331, name="adj-small-hll")
    geo = oracle.build_geometry(w.x)
    srcs = oracle.build_sources(geo, w.xs)
    tab = oracle.hll_table()
    ts = TorchStep(geo, srcs, hll=tab)
    g = workloads.rng(332)
    probes = np.sort(g.choice(w.n, 64, replace=False))
    Et = g.lognormal(size=(64, w.groups))
    return w, geo, srcs, ts, probes, Et, tab


def loss_np_hll(geo, srcs, U0, L, steps, probes, Et, tab):
    U, _ = oracle.run(geo, srcs, U0, L, steps, hll=tab)
    return float(((U[probes, :, 0] - Et) ** 2).sum())


def test_hll_forward_matches_oracle(small_hll):
    w, geo, srcs, ts, _, _, tab = small_hll
    ref, _ = oracle.run(geo, srcs, w.U0, w.L, 3, hll=tab)
    got = ts.run(torch.from_numpy(w.U0), torch.from_numpy(w.L), geo.dt, 3).numpy()
    scale = np.abs(ref).max(axis=-1, keepdims=True)
    assert (np.abs(got - ref) / scale).max() < 1e-12
    glf, _ = oracle.run(geo, srcs, w.U0, w.L, 3)
    assert (np.abs(got - glf) / scale).max() > 1e-6          # the solver matters here


def test_hll_autograd_matches_finite_differences(small_hll):
    w, geo, srcs, ts, probes, Et, tab = small_hll
    U0 = torch.from_numpy(w.U0.copy()).requires_grad_(True)
    L = torch.from_numpy(w.L.copy()).requires_grad_(True)
    U = ts.run(U0, L, geo.dt, w.steps)
    loss = ((U[probes, :, 0] - torch.from_numpy(Et)) ** 2).sum()
    gL, gU = torch.autograd.grad(loss, (L, U0))
    gL, gU = gL.numpy(), gU.numpy()
    for s in range(w.L.shape[0]):
        for grp in range(w.groups):
            def f(v):
                Lx = w.L.copy()
                Lx[s, grp] = v
                return loss_np_hll(geo, srcs, w.U0, Lx, w.steps, probes, Et, tab)
            ok, fds = fd_matches(f, w.L[s, grp], gL[s, grp], w.L[s, grp])
            assert ok, (s, grp, gL[s, grp], fds)
    g = workloads.rng(17)
    for _ in range(12):
        i = int(g.choice(probes))
        grp, m = int(g.integers(w.groups)), int(g.integers(4))

        def f(v):
            Ux = w.U0.copy()
            Ux[i, grp, m] = v
            return loss_np_hll(geo, srcs, Ux, w.L, w.steps, probes, Et, tab)
        ok, fds = fd_matches(f, w.U0[i, grp, m], gU[i, grp, m], np.abs(w.U0[i, grp]).max())
        assert ok, (i, grp, m, gU[i, grp, m], fds)


# ---------------------------------------------------------------------------
# The Ivanova surfaces (Part II eq:IvanovaAij): forward against the C
# oracle's transport with those surfaces, autograd against its central
# differences in the luminosities.
def test_ivanova_forward_and_gradient():
    w = workloads.lattice_workload(9, 2, 3, 3, seed=341, name="adj-small-iva")
    geo = oracle.build_geometry(w.x)
    srcs = oracle.build_sources(geo, w.xs)
    ts = TorchStep(geo, srcs, ivanova=True)
    ref, _ = oracle.run(geo, srcs, w.U0, w.L, 3, ivanova=True)
    got = ts.run(torch.from_numpy(w.U0), torch.from_numpy(w.L), geo.dt, 3).numpy()
    scale = np.abs(ref).max(axis=-1, keepdims=True)
    assert (np.abs(got - ref) / scale).max() < 1e-12
    hop, _ = oracle.run(geo, srcs, w.U0, w.L, 3)
    assert (np.abs(got - hop) / scale).max() > 1e-6
    g = workloads.rng(342)
    probes = np.sort(g.choice(w.n, 48, replace=False))
    Et = g.lognormal(size=(48, w.groups))
    L = torch.from_numpy(w.L.copy()).requires_grad_(True)
    U = ts.run(torch.from_numpy(w.U0), L, geo.dt, 3)
    (gL,) = torch.autograd.grad(((U[probes, :, 0] - torch.from_numpy(Et)) ** 2).sum(), (L,))
    gL = gL.numpy()
    for s in range(w.L.shape[0]):
        for grp in range(w.groups):
            def f(v):
                Lx = w.L.copy()
                Lx[s, grp] = v
                U, _ = oracle.run(geo, srcs, w.U0, Lx, 3, ivanova=True)
                return float(((U[probes, :, 0] - Et) ** 2).sum())
            ok, fds = fd_matches(f, w.L[s, grp], gL[s, grp], w.L[s, grp])
            assert ok, (s, grp, gL[s, grp], fds)
