"""The transport's algorithmic flop count, as the roofline takes it, against
an instrumented count of an independent formulation.

bench.transport_flops_per_pair(G) = 74 + 179 G is the count of the kernel's
own arithmetic per pair flux evaluation (fma = 2).  Here every floating-point
operation of the differentiable torch reference's transport (oracle/torch_ref,
written from the thesis' equations, not from the kernel) is counted by a torch
dispatch mode, per neighbour entry: the per-group part from the difference
between G = 2 and G = 1 (extrapolation, limiter, face guards, both M1 fluxes,
GLF, accumulation), the pair geometry from the constructor's surfaces
(counted on two particle sets to separate the gather entries from the pair
entries).  Comparisons, selections, min/max and absolute values count zero.
The two formulations differ in detail (the reference forms the minmod sign
from a product, raises to powers, divides where the kernel multiplies, and
recomputes per entry the per-particle factors sigma/H^3, V and 1/h that the
kernel reads from the geometry record), so the bounds are loose: 10% per
group (measured 188.4 against 179) and 60-100% for the pair geometry
(measured 106 against 74); a mistake in the formula (a missing group factor,
a term counted twice) moves it far beyond them.
"""
import numpy as np
import torch
from torch.utils._python_dispatch import TorchDispatchMode

import oracle
import workloads
from bench import transport_flops_per_pair
from oracle.torch_ref import TorchStep

ELEMENTWISE = {"add", "sub", "rsub", "mul", "div", "neg", "sqrt", "rsqrt", "reciprocal"}


class FlopCount(TorchDispatchMode):
    def __init__(self):
        super().__init__()
        self.flops = 0

    def __torch_dispatch__(self, func, types, args=(), kwargs=None):
        out = func(*args, **(kwargs or {}))
        name = func.__name__.split(".")[0]
        if name in ELEMENTWISE:
            self.flops += out.numel()
        elif name == "pow":                      # x ** 3: two products
            self.flops += 2 * out.numel()
        elif name == "sum":
            self.flops += args[0].numel() - out.numel()
        elif name in ("bmm", "mm"):              # m n (2k - 1)
            a, b = args[0], args[1]
            k = a.shape[-1]
            self.flops += out.numel() * (2 * k - 1)
        elif name == "linalg_vector_norm":
            self.flops += 2 * args[0].numel()    # squares and sums, plus the root
        return out


def lattice(groups):
    w = workloads.lattice_workload(8, groups, 0, 3, seed=11, name="flops")
    return w, oracle.build_geometry(w.x)


def transport_flops(groups):
    w, geo = lattice(groups)
    ts = TorchStep(geo)
    U = torch.from_numpy(w.U0.copy())
    D = ts.gradient(U)
    with FlopCount() as fc:
        ts.transport(U, D, geo.dt)
    return fc.flops, ts.sk.numel()


def test_per_group_count():
    f1, e1 = transport_flops(1)
    f2, e2 = transport_flops(2)
    assert e1 == e2
    per_group = (f2 - f1) / e1
    formula = transport_flops_per_pair(2) - transport_flops_per_pair(1)
    print(f"per group and entry: instrumented {per_group:.1f}, formula {formula}")
    assert abs(per_group / formula - 1) < 0.10


def test_pair_geometry_count():
    rows = []
    for w in (lattice(1)[0], workloads.config(2, scale=(1 << 11) / (1 << 22))):
        geo = oracle.build_geometry(w.x)
        with FlopCount() as fc:
            TorchStep(geo)
        rows.append((geo.gptr[-1], geo.sptr[-1], fc.flops))
    a = np.array([[r[0], r[1]] for r in rows], dtype=float)
    per_gather, per_pair = np.linalg.solve(a, np.array([r[2] for r in rows], dtype=float))
    formula = transport_flops_per_pair(0)
    print(f"pair geometry per entry: instrumented {per_pair:.1f}, formula {formula}; "
          f"gather weights {per_gather:.1f}")
    assert 0.6 < formula / per_pair <= 1.0
