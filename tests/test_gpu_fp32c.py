"""Compensated-FP32 path against the FP64 oracle.

The target is 1e-5 relative on E and F per state: every case asserts it for
every state, relative to the state's own magnitude max(E, |F|/c) (floored at
1e-6 of the mean energy), and reports the distribution (measured maxima
1.4e-7 on the lattice over 10 steps, 4.8e-7 on the lattice with sources and
7.0e-7 on the clustered set over 5 steps).  An FP32 pair flux carries about
1e-7 of the brighter state of its pair, so a faint state next to a bright one
inherits error relative to the bright one; the error against the local scale
max(E, |F|/c) over the particle and its neighbours is asserted too.  Over
many steps of a large clustered set a few faint states do exceed 1e-5 (the
benchmark's 2^22-particle leg reports how many).  Photon totals against the
oracle's FP64 totals.
"""
import numpy as np
import pytest
import torch

import oracle
import workloads
from tests.gpu_util import dev, err_summary, local_err, log, state_err, unsort

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_2302_12727_amd import RT  # noqa: E402

TOL32 = 1e-5


def per_state(got, ref, floor_frac=1e-6):
    """Error of (E, F) of every state relative to its own magnitude
    max(E, |F|/c), floored at floor_frac times the mean energy."""
    scale = np.maximum(np.abs(ref).max(axis=-1), floor_frac * np.abs(ref[..., 0]).mean())
    return np.abs(got - ref).max(axis=-1) / scale


def report(name, got, ref):
    per = per_state(got, ref)
    q = np.quantile(per, [0.5, 0.99, 0.999, 1.0])
    above = int((per > TOL32).sum())
    log(f"{name}: per-state rel err median {q[0]:.2e} p99 {q[1]:.2e} p99.9 {q[2]:.2e} "
        f"max {q[3]:.2e}; {above} of {per.size} states above {TOL32:g}")
    return per


def run32(w, steps, geo_h=None):
    rt = RT(w.n, w.groups, precision="fp32c")
    perm, h, V, dt = rt.rt_build_cells(dev(w.x), None if geo_h is None else dev(geo_h))
    if w.xs.shape[0]:
        rt.rt_set_sources(dev(w.xs))
    p = perm.cpu().numpy()
    U = dev(w.U0[p]).float()
    L = dev(w.L) if w.xs.shape[0] else None
    Q = torch.zeros(w.groups, dtype=torch.float64, device="cuda")
    for _ in range(steps):
        U = rt.step(U, L, photon_total=Q)
    rt.rt_sync()
    return unsort(U.double().cpu().numpy(), p), Q.cpu().numpy(), rt, p


def test_fp32c_gradient_close():
    w = workloads.config(0)
    geo = oracle.build_geometry(w.x)
    rt = RT(w.n, w.groups, precision="fp32c")
    perm, *_ = rt.rt_build_cells(dev(w.x))
    p = perm.cpu().numpy()
    UD = rt.rt_gradient(dev(w.U0[p]).float())
    got = unsort(rt.gradients_of(UD).double().cpu().numpy(), p)
    ref = oracle.gradient(geo, w.U0)
    scale = np.abs(ref).max(axis=(-1, -2), keepdims=True)
    err = (np.abs(got - ref) / scale).max()
    log(f"fp32c gradient max rel err {err:.3e}")
    assert err < 1e-5


def test_fp32c_gradient_union_and_staged_blocks():
    """The FP32C gradient reads a block's neighbours from their union staged in
    LDS where it fits (576 rows at 4 groups) and stages rows per pair in the
    other blocks: a 4-group Plummer set takes both paths."""
    w = workloads.config(4, scale=(1 << 14) / (1 << 24))   # Plummer + background, 4 groups
    log(f"case plummer n={w.n} G={w.groups}: fp32c gradient union and staged blocks")
    geo = oracle.build_geometry(w.x)
    rt = RT(w.n, w.groups, precision="fp32c")
    perm, *_ = rt.rt_build_cells(dev(w.x), dev(geo.h))
    p = perm.cpu().numpy()
    st = rt.rt_get_stats()
    log(f"fp32c blocks from the union: {st['union_blocks']}, staged: {st['union_staged_blocks']}")
    assert st["union_blocks"] > 0 and st["union_staged_blocks"] > 0
    assert st["union_blocks"] + st["union_staged_blocks"] == (w.n + 63) // 64
    UD = rt.rt_gradient(dev(w.U0[p]).float())
    rt.rt_sync()
    got = unsort(rt.gradients_of(UD).double().cpu().numpy(), p)
    ref = oracle.gradient(geo, w.U0)
    scale = np.abs(ref).max(axis=(-1, -2), keepdims=True)
    err = (np.abs(got - ref) / scale).max()
    log(f"fp32c union gradient max rel err {err:.3e}")
    assert err < 1e-5
    assert np.array_equal(unsort(rt.states_of(UD).cpu().numpy(), p), w.U0.astype(np.float32))


def test_fp32c_gradient_paths_identical_bits():
    """The union kernel sums every component in the same order as one lane per
    particle (the staged kernel), so a block gives identical bits on either
    path.  Groups do not mix in the gradient, so group g of a 4-group run
    equals a 1-group run on group g's states; a 1-group union holds 1024 rows
    against 576 at 4 groups, so blocks between the two take the union path in
    one run and the staged path in the other."""
    w = workloads.config(4, scale=(1 << 14) / (1 << 24))   # Plummer + background, 4 groups
    geo = oracle.build_geometry(w.x)
    rt4 = RT(w.n, 4, precision="fp32c")
    perm4, *_ = rt4.rt_build_cells(dev(w.x), dev(geo.h))
    s4 = rt4.rt_get_stats()
    U = dev(w.U0[perm4.cpu().numpy()]).float()
    G4 = rt4.gradients_of(rt4.rt_gradient(U)).cpu().numpy()
    switched = 0
    for g in range(4):
        rt1 = RT(w.n, 1, precision="fp32c")
        perm1, *_ = rt1.rt_build_cells(dev(w.x), dev(geo.h))
        assert torch.equal(perm1, perm4)
        s1 = rt1.rt_get_stats()
        switched = s1["union_blocks"] - s4["union_blocks"]
        G1 = rt1.gradients_of(rt1.rt_gradient(U[:, g:g + 1].contiguous())).cpu().numpy()
        assert np.array_equal(G1[:, 0].view(np.uint32), G4[:, g].view(np.uint32)), g
        del rt1
    log(f"fp32c gradient paths: 4 groups {s4['union_blocks']} union / {s4['union_staged_blocks']} "
        f"staged; {switched} blocks on the union path only at 1 group; identical bits")
    assert switched > 0


def test_fp32c_lattice16_ten_steps():
    w = workloads.config(0)
    geo = oracle.build_geometry(w.x)
    ref, _ = oracle.run(geo, None, w.U0, None, w.steps)
    got, Q, _, _ = run32(w, w.steps)
    err = state_err(got, ref)
    Qo = oracle.photon_total(geo, ref)
    log("fp32c lattice16 10 steps: " + err_summary(got, ref, geo.sptr, geo.sidx) +
        f"; photon total rel {np.abs(Q / Qo - 1).max():.3e}")
    per = report("fp32c lattice16 10 steps", got, ref)
    assert per.max() <= TOL32
    assert err < TOL32
    assert np.allclose(Q, Qo, rtol=1e-6)


def test_fp32c_plummer_with_source():
    w = workloads.config(2, scale=(1 << 15) / (1 << 22))
    geo = oracle.build_geometry(w.x)
    srcs = oracle.build_sources(geo, w.xs)
    ref, _ = oracle.run(geo, srcs, w.U0, w.L, 5)
    got, Q, _, _ = run32(w, 5)
    log("fp32c plummer 5 steps: " + err_summary(got, ref, geo.sptr, geo.sidx))
    per = report("fp32c plummer 5 steps", got, ref)
    assert per.max() <= TOL32
    assert local_err(got, ref, geo.sptr, geo.sidx) < TOL32
    assert np.allclose(Q, oracle.photon_total(geo, ref), rtol=1e-6)


def test_fp32c_mid_lattice_sources():
    w = workloads.config(1, scale=(20 ** 3) / (128 ** 3))
    geo = oracle.build_geometry(w.x)
    srcs = oracle.build_sources(geo, w.xs)
    ref, _ = oracle.run(geo, srcs, w.U0, w.L, 5)
    got, Q, _, _ = run32(w, 5)
    log("fp32c lattice20 S=16 5 steps: " + err_summary(got, ref, geo.sptr, geo.sidx))
    per = report("fp32c lattice20 S=16 5 steps", got, ref)
    assert per.max() <= TOL32
    assert local_err(got, ref, geo.sptr, geo.sidx) < TOL32
    assert np.allclose(Q, oracle.photon_total(geo, ref), rtol=1e-6)


@pytest.mark.parametrize("n_side,groups", [(9, 1), (11, 2), (7, 3)])
def test_fp32c_ragged_sizes(n_side, groups):
    """The compensated-FP32 tile transport and union gradient at 1-3 groups on
    lattices whose last tile is partial (729, 1331 and 343 particles), with
    sources, against the oracle."""
    w = workloads.lattice_workload(n_side, groups, 2, 3, seed=920 + n_side, name="ragged32")
    log(f"case fp32c ragged lattice{n_side} G={groups} n={w.n}")
    geo = oracle.build_geometry(w.x)
    srcs = oracle.build_sources(geo, w.xs)
    ref, _ = oracle.run(geo, srcs, w.U0, w.L, 3)
    got, Q, _, _ = run32(w, 3)
    per = report(f"fp32c ragged lattice{n_side} G={groups} 3 steps", got, ref)
    assert per.max() <= TOL32
    assert np.allclose(Q, oracle.photon_total(geo, ref), rtol=1e-6)
