"""The large adjoint configuration at reduced particle count: the Plummer +
background mix with 4 groups and 256 sources at random particles, 8192
particles instead of 2^24.

- The full recipe (50 steps, checkpoints every 10, loss on the probes against
  a target from perturbed luminosities): the compensated-FP32 adjoint against
  the FP64 adjoint, both through the library's rollout (dL 1e-4 normwise, the
  bound of the small FP32C adjoint case; measured 9e-6; dU0 1e-5 of the
  largest entry for 99% of the entries).
- A short rollout (6 steps, checkpoints every 3) of the same set: the FP64
  adjoint against the differentiable torch reference (1e-9), which is itself
  pinned to the C oracle and to finite differences.
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
from paper_2302_12727_amd.rollout import RolloutBuffers, rollout  # noqa: E402

N = 8192


@pytest.fixture(scope="module")
def c5small():
    w = workloads.config(4, scale=N / (1 << 24))
    assert w.n == N and w.groups == 4 and w.xs.shape[0] == 256
    log(f"case C5 at reduced size: plummer n={w.n} G={w.groups} S={w.xs.shape[0]} "
        f"steps {w.steps} ckpt {w.ckpt_every}")
    geo = oracle.build_geometry(w.x)
    srcs = oracle.build_sources(geo, w.xs)
    return w, geo, srcs


def context(w, geo, precision):
    rt = RT(w.n, w.groups, precision=precision, cfl=w.cfl, c_red=w.c_red)
    perm, *_ = rt.rt_build_cells(dev(w.x), dev(geo.h))
    rt.rt_set_sources(dev(w.xs))
    rt.rt_sync()
    return rt, perm.cpu().numpy()


def rel(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


def gpu_gradients(rt, p, w, steps, ckpt, Et, bufs=None):
    inv = np.empty_like(p)
    inv[p] = np.arange(w.n)
    pr = torch.as_tensor(inv[w.probes], device="cuda")
    U0 = dev(w.U0[p]).to(rt.sdtype).requires_grad_(True)
    L = dev(w.L).requires_grad_(True)
    U = rollout(rt, L, U0, steps, ckpt_every=ckpt, bufs=bufs)
    loss = ((U[pr, :, 0].double() - dev(Et)) ** 2).sum()
    loss.backward()
    rt.rt_sync()
    return float(loss), unsort(U0.grad.double().cpu().numpy(), p), L.grad.cpu().numpy()


def target(rt, p, w, steps, ckpt):
    inv = np.empty_like(p)
    inv[p] = np.arange(w.n)
    with torch.no_grad():
        Ut = rollout(rt, dev(w.L_target), dev(w.U0[p]).to(rt.sdtype), steps, ckpt)
    return Ut[torch.as_tensor(inv[w.probes], device="cuda"), :, 0].double().cpu().numpy()


def test_c5_recipe_fp32c_adjoint_against_fp64(c5small):
    w, geo, _ = c5small
    rt64, p = context(w, geo, "fp64")
    rt32, p32 = context(w, geo, "fp32c")
    assert np.array_equal(p, p32)
    Et = target(rt64, p, w, w.steps, w.ckpt_every)
    l64, gU64, gL64 = gpu_gradients(rt64, p, w, w.steps, w.ckpt_every, Et)
    bufs = RolloutBuffers(rt32, w.steps, w.ckpt_every)
    l32, gU32, gL32 = gpu_gradients(rt32, p, w, w.steps, w.ckpt_every, Et, bufs=bufs)
    # the same rollout again through the same buffers gives the same bits
    l32b, gU32b, gL32b = gpu_gradients(rt32, p, w, w.steps, w.ckpt_every, Et, bufs=bufs)
    assert l32b == l32 and np.array_equal(gU32b, gU32) and np.array_equal(gL32b, gL32)
    d = np.abs(gU32 - gU64) / np.abs(gU64).max()
    q = np.quantile(d, [0.5, 0.99, 0.999])
    eL = rel(gL32, gL64)
    log(f"C5 recipe at n={w.n}: loss fp64 {l64:.6e} fp32c {l32:.6e}; fp32c vs fp64 adjoint: "
        f"dL {eL:.2e} normwise, dU0 median {q[0]:.1e} p99 {q[1]:.1e} p99.9 {q[2]:.1e} "
        f"max {d.max():.1e}")
    assert abs(l32 / l64 - 1) < 1e-4
    assert eL < 1e-4
    assert q[1] < 1e-5


def test_c5_short_rollout_fp64_adjoint_against_torch_reference(c5small):
    w, geo, srcs = c5small
    steps, ckpt = 6, 3
    rt, p = context(w, geo, "fp64")
    Et = target(rt, p, w, steps, ckpt)
    ts = TorchStep(geo, srcs)
    U0 = torch.from_numpy(w.U0.copy()).requires_grad_(True)
    L = torch.from_numpy(w.L.copy()).requires_grad_(True)
    U = ts.run(U0, L, geo.dt, steps)
    loss = ((U[w.probes, :, 0] - torch.from_numpy(Et)) ** 2).sum()
    gU_ref, gL_ref = torch.autograd.grad(loss, (U0, L))
    lg, gU, gL = gpu_gradients(rt, p, w, steps, ckpt, Et)
    e1, e2 = rel(gU, gU_ref.numpy()), rel(gL, gL_ref.numpy())
    st = rt.rt_get_stats()
    log(f"C5 set, {steps}-step rollout: loss {lg:.6e} (reference {float(loss):.6e}); "
        f"dU0 rel err {e1:.2e}, dL rel err {e2:.2e}; transposed gradient: "
        f"{st['adj_union_blocks']} blocks from the union, {st['adj_union_staged_blocks']} staged")
    # the clustered set takes both paths of the transposed gradient
    assert st["adj_union_blocks"] > 0 and st["adj_union_staged_blocks"] > 0
    assert st["adj_union_blocks"] + st["adj_union_staged_blocks"] == (w.n + 63) // 64
    assert lg == pytest.approx(float(loss), rel=1e-12)
    assert e1 < 1e-9 and e2 < 1e-9
