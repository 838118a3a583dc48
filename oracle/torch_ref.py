"""Differentiable FP64 replica of the RT step in plain torch (CPU) -- TEST
INFRASTRUCTURE ONLY.

The thesis has no adjoint.  This module gives the reference gradient for the
HIP adjoint: it evaluates the same step as the C oracle (Part III "One RT
time step": injection, least-squares gradient, transport with minmod, face
guards, M1 closure, GLF, post-update guard) with torch operations vectorised
over the oracle's neighbour entries, so that autograd differentiates it.  Its
forward is pinned to the C oracle (to rounding) and its gradients to central
finite differences of the C oracle (tests/test_adjoint_ref.py).

The M1 flux through the effective surface A is written with g = F/E
(c^2 P A = c^2 E (1-chi)/2 A + 3/(2+sqrt(4-3f^2)) (g.A) F), which avoids the
0/0 of n = F/|F| and its infinite derivative at F = 0.  Geometry (h, V, B,
surfaces) is static and not differentiated.
"""
from __future__ import annotations

import numpy as np
import torch

SIGMA3 = 16.0 / np.pi


def _w(q):
    a = torch.clamp(1.0 - q, min=0.0)
    b = torch.clamp(0.5 - q, min=0.0)
    return a ** 3 - 4.0 * b ** 3


def guard(q: torch.Tensor, c: float) -> torch.Tensor:
    """E < 0 -> 0 (and F = 0); E = 0 -> F = 0; |F| > cE -> F scaled to cE."""
    E = q[..., 0]
    F = q[..., 1:]
    E = torch.where(E < 0, torch.zeros_like(E), E)
    F2 = (F * F).sum(-1)
    lim = c * E
    over = F2 > lim * lim
    Fn = torch.sqrt(torch.where(over, F2, torch.ones_like(F2)))
    sc = torch.where(over, lim / Fn, torch.ones_like(F2))
    F = F * sc[..., None]
    F = torch.where((E == 0)[..., None], torch.zeros_like(F), F)
    return torch.cat([E[..., None], F], dim=-1)


def flux_through(q: torch.Tensor, A: torch.Tensor, c: float) -> torch.Tensor:
    """(F.A, c^2 P A) of guarded states q [..., 4] through surfaces A [..., 3]."""
    E = q[..., 0]
    F = q[..., 1:]
    pos = E > 0
    iE = torch.where(pos, 1.0 / torch.where(pos, E, torch.ones_like(E)), torch.zeros_like(E))
    g = F * iE[..., None]
    f2 = (g * g).sum(-1) / (c * c)
    s = torch.sqrt(torch.clamp(4.0 - 3.0 * f2, min=0.0))
    idv = 1.0 / (2.0 + s)
    a = c * c * E * (1.0 / 3.0 - f2 * idv)
    b = 3.0 * idv * (g * A).sum(-1)
    out0 = (F * A).sum(-1)
    outv = a[..., None] * A + b[..., None] * F
    return torch.cat([out0[..., None], outv], dim=-1)


class TorchStep:
    """One RT step on the oracle's geometry (oracle.Geometry, oracle.Sources)."""

    def __init__(self, geo, srcs=None):
        f = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64)
        n = geo.n
        self.n, self.c = n, float(geo.c)
        box = float(geo.box[0])
        x, H, V, h = f(geo.x), f(geo.H), f(geo.V), f(geo.h)
        B = f(geo.B)
        self.V = V
        # gather entries (i, j), j in G(i): psi_tilde_j(x_i) = B_i s_ij W(r_ij, H_i) V_i
        gi = torch.as_tensor(np.repeat(np.arange(n), np.diff(geo.gptr)))
        gj = torch.as_tensor(geo.gidx)
        s = x[gj] - x[gi]
        s = s - box * torch.round(s / box)
        r = torch.linalg.norm(s, dim=1)
        psi = SIGMA3 / H[gi] ** 3 * _w(r / H[gi]) * V[gi]
        self.gi, self.gj = gi, gj
        self.pt = torch.einsum("eab,eb->ea", B[gi], s) * psi[:, None]
        # symmetric entries (k, l): A_kl = V_k psi~_l(x_k) - V_l psi~_k(x_l)
        sk = torch.as_tensor(np.repeat(np.arange(n), np.diff(geo.sptr)))
        sl = torch.as_tensor(geo.sidx)
        s = x[sl] - x[sk]
        s = s - box * torch.round(s / box)
        r = torch.linalg.norm(s, dim=1)
        Wk = SIGMA3 / H[sk] ** 3 * _w(r / H[sk])
        Wl = SIGMA3 / H[sl] ** 3 * _w(r / H[sl])
        tl = torch.einsum("eab,eb->ea", B[sk], s) * (Wk * V[sk])[:, None]
        tk = torch.einsum("eab,eb->ea", B[sl], -s) * (Wl * V[sl])[:, None]
        A = V[sk][:, None] * tl - V[sl][:, None] * tk
        self.sk, self.sl, self.s, self.A = sk, sl, s, A
        self.An = torch.linalg.norm(A, dim=1)
        self.wk = h[sk] / (h[sk] + h[sl])
        self.wl = h[sl] / (h[sk] + h[sl])
        if srcs is not None and srcs.src.size:
            self.src = torch.as_tensor(srcs.src)
            self.gas = torch.as_tensor(srcs.gas)
            self.coef = f(srcs.xi) / V[self.gas]
        else:
            self.src = None

    def inject(self, U, L, dt):
        if self.src is None:
            return U
        add = torch.zeros(self.n, U.shape[1], dtype=U.dtype).index_add(
            0, self.gas, self.coef[:, None] * L[self.src])
        return torch.cat([(U[..., 0] + dt * add)[..., None], U[..., 1:]], dim=-1)

    def gradient(self, U):
        d = (U[self.gj] - U[self.gi])[..., None] * self.pt[:, None, None, :]
        return torch.zeros(self.n, U.shape[1], 4, 3, dtype=U.dtype).index_add(0, self.gi, d)

    def transport(self, U, D, dt):
        c = self.c
        s = self.s[:, None, None, :]
        dk = (D[self.sk] * s).sum(-1)
        dl = (D[self.sl] * s).sum(-1)
        m = torch.where(dk * dl > 0, torch.where(dk.abs() <= dl.abs(), dk, dl),
                        torch.zeros_like(dk))
        qL = guard(U[self.sk] + self.wk[:, None, None] * m, c)
        qR = guard(U[self.sl] - self.wl[:, None, None] * m, c)
        A = self.A[:, None, :]
        P = 0.5 * (flux_through(qL, A, c) + flux_through(qR, A, c)) \
            - 0.5 * c * self.An[:, None, None] * (qR - qL)
        acc = torch.zeros_like(U).index_add(0, self.sk, P)
        return guard(U - dt / self.V[:, None, None] * acc, c)

    def step(self, U, L, dt):
        U1 = self.inject(U, L, dt)
        return self.transport(U1, self.gradient(U1), dt)

    def run(self, U, L, dt, steps):
        for _ in range(steps):
            U = self.step(U, L, dt)
        return U
