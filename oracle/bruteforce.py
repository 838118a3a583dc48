"""All-pairs O(N^2) NumPy evaluation of the same definitions, for tiny inputs.

Test infrastructure for pinning the oracle: it shares nothing with
`rt_oracle.c` (no neighbour lists, no loops over CSR rows) and evaluates every
sum of Part II of the thesis over the full N x N matrix of minimum-image
separations.  Use only for N up to a few thousand.
"""
from __future__ import annotations

import numpy as np

SIGMA3 = 16.0 / np.pi


def kernel_w(q):
    q = np.asarray(q, dtype=np.float64)
    a = 1.0 - q
    b = 0.5 - q
    inner = a ** 3 - 4.0 * b ** 3
    outer = a ** 3
    return np.where(q <= 0.5, inner, np.where(q < 1.0, outer, 0.0))


def kernel_W(r, H):
    return SIGMA3 / H ** 3 * kernel_w(r / H)


def separations(x, box=1.0):
    """s[i, j] = x_j - x_i wrapped to the nearest image."""
    s = x[None, :, :] - x[:, None, :]
    s -= box * np.rint(s / box)
    return s


def smoothing_lengths(x, eta, kappa, box=1.0, iters=64):
    """Bisection on h^3 sum_j W(r_ij, kappa h) = eta^3 over all particles."""
    r = np.linalg.norm(separations(x, box), axis=2)
    n = x.shape[0]
    lo = np.zeros(n)
    hi = np.full(n, 0.5 * box / kappa)
    for _ in range(iters):
        mid = 0.5 * (lo + hi)
        g = mid ** 3 * kernel_W(r, kappa * mid[:, None]).sum(axis=1) - eta ** 3
        lo = np.where(g < 0, mid, lo)
        hi = np.where(g < 0, hi, mid)
    return 0.5 * (lo + hi)


def geometry(x, H, box=1.0):
    s = separations(x, box)
    r = np.linalg.norm(s, axis=2)
    Wm = kernel_W(r, H[:, None])                   # W(r_ij, H_i), includes self
    omega = Wm.sum(axis=1)
    V = 1.0 / omega
    psi = Wm / omega[:, None]                      # psi_j(x_i)
    E = np.einsum("ija,ijb,ij->iab", s, s, psi)
    B = np.linalg.inv(E)
    gather = (r < H[:, None]) & ~np.eye(x.shape[0], dtype=bool)
    sym = gather | gather.T
    return dict(s=s, r=r, omega=omega, V=V, psi=psi, E=E, B=B, gather=gather, sym=sym)


def psitilde(geo):
    """psit[i, j, a] = psi_tilde_j^a(x_i)."""
    return np.einsum("iab,ijb,ij->ija", geo["B"], geo["s"], geo["psi"])


def gradient(geo, U):
    """dU[i, g, q, a] = sum_j (U_j - U_i) psi_tilde_j^a(x_i)."""
    pt = psitilde(geo)
    d = U[None, :, :, :] - U[:, None, :, :]       # [i, j, g, q]
    return np.einsum("ijgq,ija->igqa", d, pt)


def surfaces(geo):
    """A[k, l] = V_k psi_tilde_l(x_k) - V_l psi_tilde_k(x_l)."""
    pt = psitilde(geo)
    V = geo["V"]
    return V[:, None, None] * pt - V[None, :, None] * np.transpose(pt, (1, 0, 2))
