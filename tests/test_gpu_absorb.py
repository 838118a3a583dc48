"""Photon removal of the thermochemistry step on the GPU (Part III "Third
step: Thermochemistry") against the oracle's, element by element.

FP64: 1e-12 per state (the same factor up to the rounding of the sum over
species); photon totals and absorbed energy 1e-12.  FP32C: the factor in
FP64 applied to FP32 states, 1e-6 per state.  Cases: a lattice with and
without densities at the end of the step, every G and several J, the clamp,
and the 2^21-particle 128^3 lattice at full size (the states do not depend on
the volumes, so the oracle runs on all of them there).
"""
import ctypes
import types

import numpy as np
import pytest
import torch

import oracle
import workloads
from tests.gpu_util import dev, log, state_err, unsort

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_2302_12727_amd import RT, RTError  # noqa: E402


def densities(n, J, seed):
    g = workloads.rng(seed)
    n_old = g.uniform(0.0, 1.0, size=(n, J))
    n_new = n_old * g.uniform(0.2, 1.0, size=(n, J))
    return n_old, n_new


def gpu_absorb(w, n_old, n_new, sigma, dt, precision="fp64"):
    rt = RT(w.n, w.groups, precision=precision)
    perm, *_ = rt.rt_build_cells(dev(w.x))
    p = perm.cpu().numpy()
    U = dev(w.U0[p]).to(rt.sdtype)
    Q = torch.zeros(w.groups, dtype=torch.float64, device="cuda")
    A = torch.zeros(w.groups, dtype=torch.float64, device="cuda")
    dtt = torch.tensor([dt], dtype=torch.float64, device="cuda")
    rt.rt_absorb(U, dev(n_old[p]), dev(sigma), n_new=None if n_new is None else dev(n_new[p]),
                 dt=dtt, photon_total=Q, absorbed=A)
    rt.rt_sync()
    return unsort(U.double().cpu().numpy(), p), Q.cpu().numpy(), A.cpu().numpy()


@pytest.mark.parametrize("with_new", [False, True])
def test_lattice_fp64(with_new):
    w = workloads.lattice_workload(16, 3, 0, 1, seed=71, name="absorb16")
    geo = oracle.build_geometry(w.x)
    n_old, n_new = densities(w.n, 3, 72)
    sigma = np.array([[0.3, 0.0, 0.0], [0.06, 0.45, 0.0], [0.008, 0.12, 0.11]])
    nn = n_new if with_new else None
    got, Q, A = gpu_absorb(w, n_old, nn, sigma, 0.4)
    ref, absorbed = oracle.absorb(geo, w.U0, n_old, sigma, 0.4, n_new=nn)
    err = state_err(got, ref)
    log(f"absorb lattice16 G=3 J=3 n_new={with_new}: max state err {err:.2e}")
    assert err < 1e-12
    assert np.allclose(Q, oracle.photon_total(geo, ref), rtol=1e-12, atol=0)
    assert np.allclose(A, absorbed, rtol=1e-12, atol=0)


@pytest.mark.parametrize("G,J", [(1, 1), (2, 3), (4, 2), (5, 8), (8, 6)])
def test_groups_and_species(G, J):
    w = workloads.lattice_workload(9, G, 0, 1, seed=80 + G, name="absorb9")
    geo = oracle.build_geometry(w.x)
    n_old, n_new = densities(w.n, J, 90 + J)
    sigma = workloads.rng(100 + G * J).uniform(0.0, 0.6, size=(G, J))
    got, Q, A = gpu_absorb(w, n_old, n_new, sigma, 0.7)
    ref, absorbed = oracle.absorb(geo, w.U0, n_old, sigma, 0.7, n_new=n_new)
    assert state_err(got, ref) < 1e-12
    assert np.allclose(A, absorbed, rtol=1e-12, atol=0)


def test_clamp():
    w = workloads.lattice_workload(7, 2, 0, 1, seed=111, name="clamp")
    geo = oracle.build_geometry(w.x)
    n_old = np.full((w.n, 1), 50.0)
    n_old[::3] = 0.0                                  # a third untouched
    sigma = np.array([[1.0], [0.01]])
    got, Q, A = gpu_absorb(w, n_old, None, sigma, 1.0)
    ref, absorbed = oracle.absorb(geo, w.U0, n_old, sigma, 1.0)
    assert state_err(got, ref) < 1e-12
    assert not got[1::3, 0].any() and np.array_equal(got[::3], w.U0[::3])
    assert np.allclose(A, absorbed, rtol=1e-12)


def test_fp32c():
    w = workloads.lattice_workload(12, 3, 0, 1, seed=121, name="absorb32")
    geo = oracle.build_geometry(w.x)
    n_old, n_new = densities(w.n, 3, 122)
    sigma = np.array([[0.3, 0.0, 0.0], [0.06, 0.45, 0.0], [0.008, 0.12, 0.11]])
    got, Q, A = gpu_absorb(w, n_old, n_new, sigma, 0.4, precision="fp32c")
    # the oracle from the FP32-rounded initial state
    ref, absorbed = oracle.absorb(geo, w.U0.astype(np.float32).astype(np.float64), n_old, sigma,
                                  0.4, n_new=n_new)
    err = state_err(got, ref)
    log(f"absorb FP32C: max state err {err:.2e}")
    assert err < 1e-6
    assert np.allclose(A, absorbed, rtol=1e-5)


def test_full_size_lattice128():
    w = workloads.config(1)                           # 128^3 jittered lattice, 3 groups
    log(f"absorb full size n={w.n} G={w.groups}")
    n_old, n_new = densities(w.n, 3, 131)
    sigma = np.array([[0.3, 0.0, 0.0], [0.06, 0.45, 0.0], [0.008, 0.12, 0.11]])
    got, Q, A = gpu_absorb(w, n_old, n_new, sigma, 0.4)
    # the updated states do not involve the volumes: unit volumes for the oracle
    stub = types.SimpleNamespace(V=np.ones(w.n), c=w.c_red)
    ref, _ = oracle.absorb(stub, w.U0, n_old, sigma, 0.4, n_new=n_new)
    err = state_err(got, ref)
    log(f"absorb full size: max state err {err:.2e}")
    assert err < 1e-12
    assert (A > 0).all() and (Q > 0).all()


def test_refusals():
    w = workloads.lattice_workload(7, 2, 0, 1, seed=141, name="refuse")
    rt = RT(w.n, w.groups)
    rt.rt_build_cells(dev(w.x))
    U = dev(w.U0)
    with pytest.raises(RTError, match="J must be"):
        rt.rt_absorb(U, dev(np.zeros((w.n, 9))), dev(np.zeros((w.groups, 9))))
    with pytest.raises(ValueError):
        rt.rt_absorb(U, dev(np.zeros((w.n, 2))), dev(np.zeros((w.groups + 1, 2))))
    sig = dev(np.zeros((w.groups, 1)))
    vp = lambda t: ctypes.c_void_p(t.data_ptr())
    with pytest.raises(RTError, match="overlap"):         # n_old inside U: rejected, no launch
        rt._check(rt.L.rt_absorb(rt.ctx, vp(U), 1, vp(U), None, vp(sig), vp(rt.dt), None, None))
