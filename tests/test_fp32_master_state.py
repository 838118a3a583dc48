"""Where the compensated-FP32 error comes from: the FP32 state or the FP32
pair arithmetic.  The torch reference (oracle/torch_ref.py, pinned to the C
oracle) run in float32 emulates three ways to take an RT step on a clustered
Plummer + background set (4096 particles, 3 groups, one central source):

- FP32 master state, FP32 pair fluxes, per-particle sums without rounding
  error (the library's compensated-FP32 mode: Kahan sums, FP64 update);
- an FP64 master state with the same FP32 pair fluxes and exact sums (each
  step rounds the state to FP32 only as the fluxes' input);
- FP32 state and plain FP32 sums.

Against the FP64 reference, per state (max(E, |F|/c), floored at 1e-6 of the
mean energy): the FP64 master state lowers the median error (the state's own
rounding) but not the tail, which the FP32 pair fluxes set (a faint state
beside a bright one takes ~1e-7 of the bright state's flux per pair).  So an
FP64 master state would add FP64 state traffic without meeting a per-state
bar any better; the library keeps the FP32 state with compensated sums.
Measured over 100 steps of 16384 particles: 8, 8 and 10 of 49152 states
above 1e-5 (maxima 4.9e-5, 7.9e-5, 9.4e-5).
"""
import numpy as np
import torch

import oracle
import workloads
from oracle.torch_ref import TorchStep, flux_through, guard


def as_type(ts, dtype):
    t = TorchStep.__new__(TorchStep)
    t.__dict__.update(ts.__dict__)
    for a in ("pt", "s", "A", "An", "wk", "wl", "V"):
        setattr(t, a, getattr(ts, a).to(dtype))
    if ts.src is not None:
        t.coef = ts.coef.to(dtype)
    return t


def flux_sums(ts, U, D, exact):
    """sum_l Phi_kl . A_kl of every particle, fluxes in U's type, summed in
    float64 (exact) or in U's type."""
    c = ts.c
    s = ts.s[:, None, None, :]
    dk = (D[ts.sk] * s).sum(-1)
    dl = (D[ts.sl] * s).sum(-1)
    m = torch.where(dk * dl > 0, torch.where(dk.abs() <= dl.abs(), dk, dl), torch.zeros_like(dk))
    qL = guard(U[ts.sk] + ts.wk[:, None, None] * m, c)
    qR = guard(U[ts.sl] - ts.wl[:, None, None] * m, c)
    A = ts.A[:, None, :]
    P = 0.5 * (flux_through(qL, A, c) + flux_through(qR, A, c)) \
        - 0.5 * c * ts.An[:, None, None] * (qR - qL)
    if exact:
        return torch.zeros(U.shape, dtype=torch.float64).index_add(0, ts.sk, P.double())
    return torch.zeros_like(U).index_add(0, ts.sk, P)


def per_state(got, ref):
    scale = np.maximum(np.abs(ref).max(axis=-1), 1e-6 * np.abs(ref[..., 0]).mean())
    return np.abs(got - ref).max(axis=-1) / scale


def test_fp64_master_state_does_not_cut_the_tail():
    w = workloads.config(2, scale=4096 / (1 << 22))
    geo = oracle.build_geometry(w.x)
    ts = TorchStep(geo, oracle.build_sources(geo, w.xs))
    t32 = as_type(ts, torch.float32)
    L, dt, c, V = torch.from_numpy(w.L.copy()), geo.dt, ts.c, ts.V[:, None, None]
    U = torch.from_numpy(w.U0.copy())
    fp32_master, fp64_master, plain = U.float(), U.clone(), U.float()
    with torch.no_grad():
        for _ in range(20):
            U = ts.step(U, L, dt)
            U1 = t32.inject(fp32_master, L.float(), dt)
            fp32_master = guard(U1.double() - dt / V * flux_sums(t32, U1, t32.gradient(U1), True),
                                c).float()
            U1 = ts.inject(fp64_master, L, dt)
            U1f = U1.float()
            fp64_master = guard(U1 - dt / V * flux_sums(t32, U1f, t32.gradient(U1f), True), c)
            U1 = t32.inject(plain, L.float(), dt)
            plain = guard(U1 - (dt / t32.V)[:, None, None] * flux_sums(t32, U1, t32.gradient(U1),
                                                                       False), c)
    ref = U.numpy()
    q = {name: np.quantile(per_state(X.double().numpy(), ref), [0.5, 0.999])
         for name, X in (("fp32", fp32_master), ("fp64", fp64_master), ("plain", plain))}
    print({k: [f"{x:.2e}" for x in v] for k, v in q.items()})
    # all three reach FP32 accuracy in the bulk
    assert max(v[0] for v in q.values()) < 1e-7
    # the FP64 state lowers the median ...
    assert q["fp64"][0] < 0.8 * q["fp32"][0]
    # ... but not the tail, which the FP32 pair fluxes set
    assert q["fp64"][1] > 0.5 * q["fp32"][1]
