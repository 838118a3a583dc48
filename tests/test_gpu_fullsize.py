"""Full-size cases, in the launch configuration the benchmark times.

C2 (128^3 jittered lattice, 3 groups, 16 sources): the HIP path against the
FP64 oracle element by element -- smoothing lengths (1e-13 relative), the
symmetric neighbour sets (exact), the photon totals (1e-12 relative) and every
state after two whole steps (1e-12 relative per state, as in the small cases).

The same C2 lattice also carries one whole step with the HLL solver, one
with the Ivanova surfaces, and the drift correction of every state, element
by element against the oracle.

C4 (the adjoint workload: the same lattice with 64 sources, 20 steps,
checkpoints every 5, loss on 4096 probes): dLoss/dL of the adjoint rollout
against central finite differences of the GPU forward on 8 luminosities,
1e-6 relative to the largest luminosity gradient.  At this size the face and
update guards switch somewhere in the domain for perturbations of 1e-5 of a
luminosity (about 1.6 million flux rescales per step), so the loss is smooth
only piecewise at that scale: the central differences of one component then
drift by a few 1e-6 of it as the step shrinks, and a component far smaller
than the loss curvature is resolved only to that absolute level.  The
per-component errors are logged; the bound is normwise.

C3 (2^22 Plummer mix with a central source): the HIP path against the FP64
oracle element by element -- smoothing lengths solved on both sides (1e-13,
with the h-solve's candidate-list overflow path taken on the GPU), the
symmetric neighbour sets (exact, up to 96 neighbours), and every state after
two whole steps (1e-12 relative per state) -- plus what holds at any size: the
smoothing-length equation of sampled particles summed by brute force over all
particles, their neighbour sets by brute force (exact), and the photon budget
of 100 FP64 steps (1e-12 relative).
"""
import numpy as np
import pytest
import torch

import oracle
import workloads
from oracle import bruteforce
from tests.gpu_util import dev, local_err, log, state_err, unsort

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_2302_12727_amd import KAPPA, ETA, RT  # noqa: E402
from paper_2302_12727_amd.rollout import rollout  # noqa: E402


def build(w, h=None, precision="fp64"):
    rt = RT(w.n, w.groups, precision=precision, cfl=w.cfl, c_red=w.c_red)
    perm, *_ = rt.rt_build_cells(dev(w.x), None if h is None else dev(h))
    if w.xs.shape[0]:
        rt.rt_set_sources(dev(w.xs))
    rt.rt_sync()
    return rt, perm.cpu().numpy()


def state_err_per_state(got, ref):
    """Per-state error relative to max(E, |F|/c) of that state (floored at 1e-6
    of the mean energy), as state_err but not reduced."""
    scale = np.maximum(np.abs(ref).max(axis=-1), 1e-6 * np.abs(ref[..., 0]).mean())
    return np.abs(got - ref).max(axis=-1) / scale


def neighbour_keys(rt, p):
    """Sorted keys i * n + j of the symmetric lists, in input numbering."""
    ptr, idx = rt.rt_get_neighbours()
    ptr, idx = ptr.cpu().numpy(), idx.cpu().numpy()
    n = p.shape[0]
    rows = np.repeat(p, np.diff(ptr)).astype(np.int64)
    keys = rows * n + p[idx].astype(np.int64)
    keys.sort()
    return keys


@pytest.fixture(scope="module")
def c2():
    w = workloads.config(1)
    log(f"case C2 lattice128 G=3 S=16 n={w.n}: oracle geometry ...")
    geo = oracle.build_geometry(w.x)
    srcs = oracle.build_sources(geo, w.xs)
    log(f"  oracle pairs {geo.n_pairs}")
    return w, geo, srcs


def test_c2_smoothing_lengths(c2):
    w, geo, _ = c2
    rt, p = build(w)
    h = unsort(rt.h.cpu().numpy(), p)
    err = float(np.abs(h / geo.h - 1).max())
    log(f"C2 smoothing lengths: max rel diff {err:.2e}")
    assert err < 1e-13


def test_c2_two_steps_every_element(c2):
    w, geo, srcs = c2
    rt, p = build(w, h=geo.h)
    assert rt.rt_get_stats()["n_pairs"] == geo.n_pairs
    n = w.n
    ref_keys = np.repeat(np.arange(n, dtype=np.int64), np.diff(geo.sptr)) * n + geo.sidx
    assert np.array_equal(neighbour_keys(rt, p), np.sort(ref_keys))
    assert float(rt.dt.item()) == pytest.approx(geo.dt, rel=1e-13)
    U = dev(w.U0[p])
    L = dev(w.L)
    Q = torch.zeros(w.groups, dtype=torch.float64, device="cuda")
    for _ in range(2):
        U = rt.step(U, L, photon_total=Q)
    got = unsort(U.cpu().numpy(), p)
    ref = w.U0.copy()
    for _ in range(2):
        ref, _ = oracle.step(geo, srcs, ref, w.L)
    err = state_err(got, ref)
    Qo = oracle.photon_total(geo, ref)
    qerr = float(np.abs(Q.cpu().numpy() / Qo - 1).max())
    log(f"C2 two steps, {n} particles x 3 groups: max state err {err:.2e}, photon total {qerr:.2e}")
    assert err < 1e-12
    assert qerr < 1e-12


def test_c2_hll_step_every_element(c2):
    """The HLL solver (eq:riemann-HLL) at full size: one whole step."""
    w, geo, srcs = c2
    rt, p = build(w, h=geo.h)
    rt.rt_set_riemann("hll")
    U = rt.step(dev(w.U0[p]), dev(w.L))
    got = unsort(U.cpu().numpy(), p)
    ref, _ = oracle.step(geo, srcs, w.U0, w.L, hll=oracle.hll_table())
    err = state_err(got, ref)
    log(f"C2 HLL step, {w.n} particles x 3 groups: max state err {err:.2e}")
    assert err < 1e-12


def test_c2_ivanova_step_every_element(c2):
    """The Ivanova surfaces (eq:IvanovaAij) at full size: one whole step."""
    w, geo, srcs = c2
    rt, p = build(w, h=geo.h)
    rt.rt_set_surfaces("ivanova")
    U = rt.step(dev(w.U0[p]), dev(w.L))
    got = unsort(U.cpu().numpy(), p)
    ref, info = oracle.step(geo, srcs, w.U0, w.L, ivanova=True)
    # The Ivanova surfaces do not close on irregular sets, and here some updated
    # states land within rounding of E = 0, where the post-update guard may
    # clip on one side and not on the other: such a state differs by a
    # rounding-level remainder, large only against its own (near-zero) size.
    # Errors are therefore measured against each neighbourhood's scale, and
    # the states off by more than 1e-12 of their own size are counted (with
    # CFL 0.9 these surfaces leave about 1e5 states below E = 0 here).
    err = local_err(got, ref, geo.sptr, geo.sidx)
    own = state_err_per_state(got, ref)
    n_off = int((own > 1e-12).sum())
    log(f"C2 Ivanova step, {w.n} particles x 3 groups: max err {err:.2e} of the neighbourhood "
        f"scale; {n_off} states off by more than 1e-12 of their own size (largest {own.max():.2e}); "
        f"oracle E clips {info['counts'][2]}")
    assert err < 1e-12
    # about 0.3% of the ~1e5 clipped states sit within rounding of the clip
    assert n_off <= max(16, 0.01 * int(info["counts"][2]))


def test_c2_drift_every_element(c2):
    """The drift correction at full size, errors against the scale of the
    summed terms (as in the drift tests)."""
    w, geo, _ = c2
    rt, p = build(w, h=geo.h)
    dx = workloads.rng(211).uniform(-0.2 / 128, 0.2 / 128, size=(w.n, 3))
    UD = rt.rt_gradient(dev(w.U0[p]))
    got = unsort(rt.rt_drift(UD, dev(dx[p])).cpu().numpy(), p)
    dU = oracle.gradient(geo, w.U0)
    ref, _, _ = oracle.drift(geo, w.U0, dx, dU=dU)
    term = (np.abs(dU) * np.abs(dx)[:, None, None, :]).sum(-1)
    scale = np.maximum(np.maximum(np.abs(w.U0).max(-1), term.max(-1)),
                       1e-6 * np.abs(w.U0[..., 0]).mean())
    err = float((np.abs(got - ref).max(-1) / scale).max())
    log(f"C2 drift, {w.n} particles x 3 groups: max err {err:.2e}")
    assert err < 1e-12


def test_c4_gradient_vs_finite_differences():
    w = workloads.config(3)
    rt, p = build(w)
    inv = np.empty_like(p)
    inv[p] = np.arange(w.n)
    pr = torch.as_tensor(inv[w.probes], device="cuda")
    U0 = dev(w.U0[p])
    with torch.no_grad():
        Et = rollout(rt, dev(w.L_target), U0, w.steps, w.ckpt_every)[pr, :, 0].clone()

    def loss_of(L):
        with torch.no_grad():
            U = rollout(rt, L, U0, w.steps, w.ckpt_every)
            return float(((U[pr, :, 0] - Et) ** 2).sum())

    Ld = dev(w.L).requires_grad_(True)
    U = rollout(rt, Ld, U0.clone().requires_grad_(True), w.steps, w.ckpt_every)
    ((U[pr, :, 0] - Et) ** 2).sum().backward()
    gL = Ld.grad.cpu().numpy()
    picks = [(s, s % w.groups) for s in range(0, w.L.shape[0], w.L.shape[0] // 8)][:8]
    gmax = float(np.abs(gL).max())
    worst = 0.0
    for s, g in picks:
        best = np.inf
        for r in (1e-3, 1e-4, 1e-5, 1e-6):
            eps = r * w.L[s, g]
            Lp, Lm = w.L.copy(), w.L.copy()
            Lp[s, g] += eps
            Lm[s, g] -= eps
            fd = (loss_of(dev(Lp)) - loss_of(dev(Lm))) / (2 * eps)
            best = min(best, abs(fd - gL[s, g]))
        log(f"  C4 dLoss/dL[{s},{g}] = {gL[s, g]:+.6e}: vs central differences "
            f"{best / abs(gL[s, g]):.2e} of itself, {best / gmax:.2e} of max |dLoss/dL|")
        worst = max(worst, best / gmax)
    log(f"C4 full size: worst error of 8 luminosity gradients {worst:.2e} of max |dLoss/dL| "
        f"= {gmax:.3e}")
    assert worst < 1e-6


@pytest.fixture(scope="module")
def c3():
    w = workloads.config(2)
    log(f"case C3 plummer G=3 n={w.n}")
    rt, p = build(w)
    return w, rt, p


def test_c3_sampled_smoothing_lengths_and_neighbours(c3):
    w, rt, p = c3
    h = unsort(rt.h.cpu().numpy(), p)
    H = KAPPA * h
    g = workloads.rng(4242)
    # the densest and the sparsest particles, and a random sample
    order = np.argsort(h)
    sample = np.unique(np.concatenate([order[:8], order[-8:], g.choice(w.n, 48, replace=False)]))
    ptr, idx = rt.rt_get_neighbours()
    ptr, idx = ptr.cpu().numpy(), idx.cpu().numpy()
    inv = np.empty_like(p)
    inv[p] = np.arange(w.n)
    worst = 0.0
    for i in sample:
        s = w.x - w.x[i]
        s -= np.rint(s)
        r = np.sqrt((s * s).sum(axis=1))
        resid = h[i] ** 3 * bruteforce.kernel_W(r, H[i]).sum() / ETA ** 3 - 1.0
        worst = max(worst, abs(resid))
        ref = np.flatnonzero((r < np.maximum(H[i], H)) & (np.arange(w.n) != i))
        k = inv[i]
        got = np.sort(p[idx[ptr[k]:ptr[k + 1]]])
        assert np.array_equal(got, ref), i
    log(f"C3: h spans {h.max() / h.min():.1f}x; {sample.size} sampled particles: "
        f"max relative residual of h^3 sum W = eta^3: {worst:.2e}; neighbour sets exact")
    assert worst < 1e-12


def test_c3_photon_budget_hundred_steps(c3):
    w, rt, p = c3
    U = dev(w.U0[p])
    L = dev(w.L)
    Q = torch.zeros(w.groups, dtype=torch.float64, device="cuda")
    ledger = torch.zeros(w.groups, dtype=torch.float64, device="cuda")
    Q0 = rt.rt_photon_total(U).cpu().numpy()
    for _ in range(w.steps):
        U = rt.step(U, L, photon_total=Q, ledger=ledger)
    Qe = Q.cpu().numpy()
    expect = Q0 + w.steps * float(rt.dt.item()) * w.L.sum(axis=0) + ledger.cpu().numpy()
    res = float(np.abs(Qe / expect - 1).max())
    log(f"C3 100 FP64 steps: photon budget residual {res:.2e} (ledger {ledger.cpu().numpy()})")
    assert res < 1e-12


def test_c3_two_steps_every_element(c3):
    """Full-size C3 against the oracle: its 43x span of smoothing lengths,
    rows of up to 96 neighbours, and the re-walks of the h-solve whose
    candidate lists overflowed."""
    w, rt, p = c3
    log(f"C3 oracle geometry of {w.n} particles ...")
    geo = oracle.build_geometry(w.x)
    srcs = oracle.build_sources(geo, w.xs)
    st = rt.rt_get_stats()
    h = unsort(rt.h.cpu().numpy(), p)
    herr = float(np.abs(h / geo.h - 1).max())
    log(f"C3: h spans {geo.h.max() / geo.h.min():.1f}x, GPU vs oracle {herr:.2e}; "
        f"{st['h_list_overflow']} particles re-walked after a list overflow; "
        f"h iterations up to {st['h_iter_max']}; max neighbours {st['max_neighbours']}")
    assert herr < 1e-13
    assert st["h_list_overflow"] > 0
    # the step on the oracle's smoothing lengths (identical neighbour sets)
    rt2, p2 = build(w, h=geo.h)
    assert rt2.rt_get_stats()["n_pairs"] == geo.n_pairs
    n = w.n
    ref_keys = np.repeat(np.arange(n, dtype=np.int64), np.diff(geo.sptr)) * n + geo.sidx
    assert np.array_equal(neighbour_keys(rt2, p2), np.sort(ref_keys))
    U = dev(w.U0[p2])
    L = dev(w.L)
    Q = torch.zeros(w.groups, dtype=torch.float64, device="cuda")
    for _ in range(2):
        U = rt2.step(U, L, photon_total=Q)
    rt2.rt_sync()
    got = unsort(U.cpu().numpy(), p2)
    del rt2
    ref = w.U0.copy()
    for _ in range(2):
        ref, _ = oracle.step(geo, srcs, ref, w.L)
    err = state_err(got, ref)
    Qo = oracle.photon_total(geo, ref)
    qerr = float(np.abs(Q.cpu().numpy() / Qo - 1).max())
    log(f"C3 two steps, {n} particles x 3 groups: max state err {err:.2e}, photon total {qerr:.2e}")
    assert err < 1e-12
    assert qerr < 1e-12
