"""rt_adjoint_static (the adjoint through the library's fixed scratch, for
callers that cannot allocate) against rt_adjoint on the same inputs: two calls
in a row on the same GPU, the second on a smaller particle set (so it runs on
whatever the first left in the shared scratch), then an FP32C call, and the
refusal of a context too large for the scratch."""
import numpy as np
import pytest
import torch

import workloads
from tests.gpu_util import dev, log

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_2302_12727_amd import RT  # noqa: E402
from paper_2302_12727_amd.rt import RT_EINVAL, RTError  # noqa: E402

TOL = {"fp64": 1e-12, "fp32c": 1e-6}


def forward_records(n_side, groups, n_src, precision, seed):
    """Context, luminosities and the forward records of one step (the gradient
    record of the injected state and the unguarded updated state)."""
    w = workloads.lattice_workload(n_side, groups, n_src, 1, seed, name="noalloc")
    rt = RT(w.n, groups, precision=precision)
    perm, *_ = rt.rt_build_cells(dev(w.x))
    rt.rt_set_sources(dev(w.xs))
    p = perm.cpu().numpy()
    U = dev(w.U0[p]).to(rt.sdtype)
    L = dev(w.L)
    rt.rt_inject(U, L)
    UD = rt.rt_gradient(U)
    Uu = torch.empty_like(U)
    rt.rt_transport(UD, U_unguarded=Uu)
    g = np.random.default_rng(seed + 7)
    lam_next = dev(g.normal(size=(w.n, groups, 4))).to(rt.sdtype)
    rt.rt_sync()
    return rt, L, UD, Uu, lam_next


def rel(a, b):
    a, b = a.double(), b.double()
    return float((a - b).abs().max() / b.abs().max().clamp_min(1e-300))


def compare(n_side, groups, n_src, precision, seed):
    rt, L, UD, Uu, lam_next = forward_records(n_side, groups, n_src, precision, seed)
    log(f"case rt_adjoint_static {precision} n={rt.n} G={groups} S={n_src}")
    dL_ref = torch.zeros((rt.S, groups), dtype=torch.float64, device="cuda")
    lam_ref = rt.rt_adjoint(None, L, lam_next, UD=UD, U_unguarded=Uu, dL_dL=dL_ref)
    dL = torch.zeros_like(dL_ref)
    lam = rt.rt_adjoint_static(L, lam_next, UD, Uu, dL_dL=dL)
    rt.rt_sync()
    e_lam, e_dL = rel(lam, lam_ref), rel(dL, dL_ref)
    log(f"  lam {e_lam:.2e} (bitwise {torch.equal(lam, lam_ref)}), dL/dL {e_dL:.2e}")
    assert e_lam <= TOL[precision] and e_dL <= TOL[precision]
    return rt


def test_two_calls_then_smaller_then_fp32c():
    compare(12, 2, 3, "fp64", 9101)
    compare(8, 2, 2, "fp64", 9102)        # smaller: reuses the first call's scratch
    compare(10, 3, 2, "fp32c", 9103)


def test_too_large_for_the_scratch_is_refused():
    # 64^3 particles x 2 groups x 4 doubles x 5 arrays = 80 MiB > 64 MiB
    rt, L, UD, Uu, lam_next = forward_records(64, 2, 1, "fp64", 9104)
    log(f"case rt_adjoint_static refusal n={rt.n}")
    lam = torch.full_like(lam_next, 7.0)
    with pytest.raises(RTError) as e:
        rt.rt_adjoint_static(L, lam_next, UD, Uu, lam=lam)
    assert e.value.code == RT_EINVAL
    assert "64" in str(e.value) or "scratch" in str(e.value)
    rt.rt_sync()
    assert bool((lam == 7.0).all())        # nothing was launched
