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

With `hll` (the wave-speed table of oracle.hll_table(), shape (NF, NMU, 2))
the transport uses the HLL solver (Part III eq:riemann-HLL) as the C oracle
does: the face states' extreme eigenvalues interpolated bilinearly in (f, mu)
from the table (which is not differentiated), and the solver's weights.  At
the kinks (the max/min of the speeds, the clamps of f and mu, the table
cells) the derivative is that of the branch the forward takes.

With `ivanova` the effective surfaces are the Ivanova ones (Part II
eq:IvanovaAij), taken pair by pair from the C oracle (static geometry, not
differentiated).
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


def hll_speeds(q: torch.Tensor, A: torch.Tensor, An: torch.Tensor, c: float,
               tab: torch.Tensor):
    """(lambda_min, lambda_max) of guarded states q [..., 4] across surfaces A
    [..., 3] (|A| = An): the table (NF, NMU, 2) at f = |F|/(cE) <= 1 and
    mu = F.A/(|F||A|) in [-1, 1], bilinear; f = mu = 0 where E or F is 0."""
    nf, nmu = tab.shape[0], tab.shape[1]
    E = q[..., 0]
    F = q[..., 1:]
    F2 = (F * F).sum(-1)
    ok = (E > 0) & (F2 > 0)
    Fn = torch.sqrt(torch.where(ok, F2, torch.ones_like(F2)))
    Es = torch.where(ok, E, torch.ones_like(E))
    fr = Fn / (c * Es)
    f = torch.where(ok, torch.where(fr <= 1.0, fr, torch.ones_like(fr)), torch.zeros_like(fr))
    mr = (F * A).sum(-1) / (Fn * An)
    mc = torch.where(mr > 1.0, torch.ones_like(mr), torch.where(mr < -1.0, -torch.ones_like(mr), mr))
    mu = torch.where(ok, mc, torch.zeros_like(mc))
    x = f * (nf - 1)
    y = (mu + 1.0) * (0.5 * (nmu - 1))
    i = torch.clamp(torch.floor(x.detach()).long(), 0, nf - 2)
    j = torch.clamp(torch.floor(y.detach()).long(), 0, nmu - 2)
    tx = (x - i)[..., None]
    ty = (y - j)[..., None]
    v = ((1 - tx) * ((1 - ty) * tab[i, j] + ty * tab[i, j + 1])
         + tx * ((1 - ty) * tab[i + 1, j] + ty * tab[i + 1, j + 1]))
    return c * v[..., 0], c * v[..., 1]


def hll_weights(loL, hiL, loR, hiR, An):
    """(w1, w2, w3) of Phi.A = w1 F_L.A + w2 F_R.A + w3 (U_R - U_L)."""
    mx = torch.where(hiL >= hiR, hiL, hiR)
    mn = torch.where(loL <= loR, loL, loR)
    lp = torch.where(mx > 0, mx, torch.zeros_like(mx))
    lm = torch.where(mn < 0, mn, torch.zeros_like(mn))
    den = lp - lm
    ok = den > 0
    iden = torch.where(ok, 1.0 / torch.where(ok, den, torch.ones_like(den)), torch.zeros_like(den))
    half = torch.full_like(den, 0.5)
    return (torch.where(ok, lp * iden, half), torch.where(ok, -lm * iden, half),
            torch.where(ok, lp * lm * An * iden, torch.zeros_like(den)))


class TorchStep:
    """One RT step on the oracle's geometry (oracle.Geometry, oracle.Sources);
    `hll` selects the HLL solver with that wave-speed table (else GLF),
    `ivanova` the Ivanova surfaces (else Hopkins)."""

    def __init__(self, geo, srcs=None, hll=None, ivanova=False):
        self.hll = None if hll is None else torch.as_tensor(np.asarray(hll, dtype=np.float64))
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
        if ivanova:
            from . import ivanova_sums, surface_ivanova
            gsum = ivanova_sums(geo)
            A = f(np.array([surface_ivanova(geo, gsum, int(k), int(l))
                            for k, l in zip(sk.numpy(), sl.numpy())]).reshape(-1, 3))
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
        if self.hll is None:
            P = 0.5 * (flux_through(qL, A, c) + flux_through(qR, A, c)) \
                - 0.5 * c * self.An[:, None, None] * (qR - qL)
        else:
            An = self.An[:, None]
            loL, hiL = hll_speeds(qL, A, An, c, self.hll)
            loR, hiR = hll_speeds(qR, A, An, c, self.hll)
            w1, w2, w3 = hll_weights(loL, hiL, loR, hiR, An)
            P = w1[..., None] * flux_through(qL, A, c) + w2[..., None] * flux_through(qR, A, c) \
                + w3[..., None] * (qR - qL)
        acc = torch.zeros_like(U).index_add(0, self.sk, P)
        return guard(U - dt / self.V[:, None, None] * acc, c)

    def step(self, U, L, dt):
        U1 = self.inject(U, L, dt)
        return self.transport(U1, self.gradient(U1), dt)

    def run(self, U, L, dt, steps):
        for _ in range(steps):
            U = self.step(U, L, dt)
        return U
