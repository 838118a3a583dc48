"""Oracle for the Gear-RT photon transport step -- TEST INFRASTRUCTURE ONLY.

A plain FP64 CPU implementation of what the HIP library computes, written from
the thesis (arXiv:2302.12727, Part II "Finite volume particle methods" and
Part III "Numerical solution strategy").  Only `tests/`, the smoke check of
`__graft_entry__` and the CPU-baseline leg of `bench.py` may import it; the
product path never does.

Layers:
  * neighbour candidates from a periodic k-d tree (scipy.spatial.cKDTree, a
    library primitive; the HIP path uses its own Morton-ordered tree);
  * per-particle arithmetic in `rt_oracle.c` (plain loops, FP64);
  * the 3x3 inversion B_i = E_i^{-1} by numpy.linalg.inv (LAPACK).

Parity status: every function is pinned by the CPU tests (closed forms of the
kernel and the M1 closure, partition of unity, linear exactness of the
gradient, lattice surfaces, the two-particle step of Appendix E, photon
conservation, brute-force sums).  The readings listed in the C file (limiter
form, face normal, guards, injection units) have no worked example in the
thesis; they are pinned only through those consequences.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
import subprocess
from typing import Optional

import numpy as np
from scipy.spatial import cKDTree

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "rt_oracle.c")
LIB = os.path.join(HERE, "liborc.so")

# H/h of the cubic spline in 3D (compact support radius over smoothing length),
# fixed by the neighbour number of eq:number-of-neighbors: (4pi/3)(kappa*eta)^3 = 48
# at eta = 1.2348.
KAPPA = 1.825742
ETA = 1.2348

RT_OK, RT_ENOCONV, RT_ESINGULAR = 0, -4, -5


class OracleError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(msg)
        self.code = code


def build(quiet: bool = True) -> str:
    """Compile rt_oracle.c into liborc.so (gcc, -O2, OpenMP, no fast-math)."""
    cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
           "-ffp-contract=off", "-o", LIB + ".tmp", SRC, "-lm"]
    subprocess.run(cmd, check=True, capture_output=quiet)
    os.replace(LIB + ".tmp", LIB)
    return LIB


_lib = None

_d = ctypes.POINTER(ctypes.c_double)
_i64 = ctypes.POINTER(ctypes.c_int64)
_i32 = ctypes.POINTER(ctypes.c_int32)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = ctypes.CDLL(LIB)
        L.orc_w.restype = ctypes.c_double
        L.orc_w.argtypes = [ctypes.c_double]
        L.orc_dw.restype = ctypes.c_double
        L.orc_dw.argtypes = [ctypes.c_double]
        L.orc_W.restype = ctypes.c_double
        L.orc_W.argtypes = [ctypes.c_double, ctypes.c_double]
        L.orc_minmod.restype = ctypes.c_double
        L.orc_minmod.argtypes = [ctypes.c_double, ctypes.c_double]
        L.orc_solve_h.restype = ctypes.c_int32
        L.orc_solve_h.argtypes = [ctypes.c_int64, ctypes.c_int32, _d, ctypes.c_double,
                                  ctypes.c_double, _d, _i32, _i32]
        L.orc_transpose.restype = None
        L.orc_transpose.argtypes = [ctypes.c_int64, _i64, _i64, _i64, _i64, _i64]
        L.orc_sym_count.restype = ctypes.c_int64
        L.orc_sym_count.argtypes = [ctypes.c_int64, _i64, _i64, _i64, _i64, _i64]
        L.orc_sym_fill.restype = None
        L.orc_sym_fill.argtypes = [ctypes.c_int64, _i64, _i64, _i64, _i64, _i64, _i64]
        L.orc_geometry.restype = None
        L.orc_geometry.argtypes = [ctypes.c_int64, _d, _d, _d, _i64, _i64, _d, _d, _d]
        L.orc_gradient.restype = None
        L.orc_gradient.argtypes = [ctypes.c_int64, ctypes.c_int32, _d, _d, _d, _d, _d,
                                   _i64, _i64, _d, _d]
        L.orc_m1_flux.restype = None
        L.orc_m1_flux.argtypes = [_d, _d, ctypes.c_double, _d]
        L.orc_glf.restype = None
        L.orc_glf.argtypes = [_d, _d, _d, ctypes.c_double, _d]
        L.orc_surface.restype = None
        L.orc_surface.argtypes = [_d, _d, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                  ctypes.c_double, _d, _d, _d, _d]
        L.orc_transport.restype = None
        L.orc_transport.argtypes = [ctypes.c_int64, ctypes.c_int32, _d, _d, _d, _d, _d, _d,
                                    _i64, _i64, ctypes.c_double, ctypes.c_double, _d, _d,
                                    _d, _i64, _d]
        L.orc_inject.restype = None
        L.orc_inject.argtypes = [ctypes.c_int64, ctypes.c_int32, _i64, _i64, _d, _d, _d,
                                 ctypes.c_double, _d]
        L.orc_source_weights.restype = ctypes.c_int32
        L.orc_source_weights.argtypes = [ctypes.c_int32, _d, _d, ctypes.c_double, _d, _d]
        L.orc_photon_total.restype = None
        L.orc_photon_total.argtypes = [ctypes.c_int64, ctypes.c_int32, _d, _d, _d]
        L.orc_dt.restype = ctypes.c_double
        L.orc_dt.argtypes = [ctypes.c_int64, _d, ctypes.c_double, ctypes.c_double]
        L.orc_num_threads.restype = ctypes.c_int32
        L.orc_num_threads.argtypes = []
        L.orc_set_num_threads.restype = None
        L.orc_set_num_threads.argtypes = [ctypes.c_int32]
        L.orc_drift.restype = None
        L.orc_drift.argtypes = [ctypes.c_int64, ctypes.c_int32, _d, _d, _d, _d, ctypes.c_double,
                                _d, _i64, _d]
        L.orc_absorb.restype = None
        L.orc_absorb.argtypes = [ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, _d, _d, _d, _d,
                                 _d, ctypes.c_double, ctypes.c_double, _d, _d]
        L.orc_hll.restype = None
        L.orc_hll.argtypes = [_d, _d, _d, ctypes.c_double, _d, ctypes.c_int32, ctypes.c_int32, _d]
        L.orc_transport_hll.restype = None
        L.orc_transport_hll.argtypes = [ctypes.c_int64, ctypes.c_int32, _d, _d, _d, _d, _d, _d,
                                        _i64, _i64, ctypes.c_double, ctypes.c_double, _d, _d,
                                        _d, _i64, _d, _d, ctypes.c_int32, ctypes.c_int32]
        L.orc_transport_ivanova.restype = None
        L.orc_transport_ivanova.argtypes = [ctypes.c_int64, ctypes.c_int32, _d, _d, _d, _d, _d,
                                            _d, _i64, _i64, ctypes.c_double, ctypes.c_double, _d,
                                            _d, _d, _i64, _d, _d, ctypes.c_int32, ctypes.c_int32,
                                            _d]
        L.orc_ivanova_sums.restype = None
        L.orc_ivanova_sums.argtypes = [ctypes.c_int64, _d, _d, _d, _i64, _i64, _d]
        L.orc_grad_psi.restype = None
        L.orc_grad_psi.argtypes = [_d, _d, ctypes.c_double, ctypes.c_double, _d, _d, _d]
        L.orc_surface_ivanova.restype = None
        L.orc_surface_ivanova.argtypes = [_d, _d, ctypes.c_double, ctypes.c_double,
                                          ctypes.c_double, ctypes.c_double, _d, _d, _d, _d]
        L.orc_bins.restype = None
        L.orc_bins.argtypes = [ctypes.c_int64, _d, ctypes.c_double, ctypes.c_double,
                               ctypes.c_double, ctypes.c_int32, _i64, _i64, _i32]
        L.orc_inject_binned.restype = None
        L.orc_inject_binned.argtypes = [ctypes.c_int64, ctypes.c_int32, _i64, _i64, _d, _d, _d,
                                        ctypes.c_double, _i32, ctypes.c_int64, _d]
        L.orc_transport_binned.restype = None
        L.orc_transport_binned.argtypes = [ctypes.c_int64, ctypes.c_int32, _d, _d, _d, _d, _d,
                                           _d, _i64, _i64, ctypes.c_double, ctypes.c_double,
                                           _i32, ctypes.c_int64, _d, _d, _d, _d, _i64, _d,
                                           _d, ctypes.c_int32, ctypes.c_int32, _d]
        _lib = L
    return _lib


def _p(a: np.ndarray, t=_d):
    return a.ctypes.data_as(t)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def _i64a(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.int64)


# ---------------------------------------------------------------------------
# scalar helpers (used by the pins)

def w(q: float) -> float:
    return lib().orc_w(q)


def dw(q: float) -> float:
    return lib().orc_dw(q)


def W(r: float, H: float) -> float:
    return lib().orc_W(r, H)


def minmod(a: float, b: float) -> float:
    return lib().orc_minmod(a, b)


def m1_flux(q, nh, c: float) -> np.ndarray:
    q, nh = _f64(q), _f64(nh)
    out = np.zeros(4)
    lib().orc_m1_flux(_p(q), _p(nh), c, _p(out))
    return out


def glf(qL, qR, nh, c: float) -> np.ndarray:
    qL, qR, nh = _f64(qL), _f64(qR), _f64(nh)
    out = np.zeros(4)
    lib().orc_glf(_p(qL), _p(qR), _p(nh), c, _p(out))
    return out


# ---------------------------------------------------------------------------
# neighbour candidates

def _knn_covering(tree: cKDTree, pts: np.ndarray, radius_fn, k0: int = 96,
                  kmax: int = 1 << 14):
    """k-nearest candidate rows for every query point such that the row
    satisfies radius_fn(rows, d, idx) (rows that fail are queried again with
    twice the k).  Returns a list of (rows, d, idx) blocks."""
    n_pts = tree.n
    out = []
    rows = np.arange(pts.shape[0])
    k = min(k0, n_pts)
    while rows.size:
        d, idx = tree.query(pts[rows], k=k, workers=-1)
        d = d.reshape(rows.size, k)
        idx = idx.reshape(rows.size, k).astype(np.int64)
        ok = radius_fn(rows, d, idx)
        if k >= n_pts:
            ok[:] = True
        out.append((rows[ok], d[ok], idx[ok]))
        rows = rows[~ok]
        if rows.size and k >= kmax:
            raise OracleError(RT_ENOCONV, "neighbour candidate set exceeds kmax")
        k = min(2 * k, n_pts)
    return out


def solve_h(tree: cKDTree, pts: np.ndarray, eta: float = ETA, kappa: float = KAPPA,
            return_blocks: bool = False):
    """Smoothing lengths of the query points over the particles in `tree`
    (eq:number-of-neighbors; root of h^3 sum_j W(r_j, kappa h) = eta^3)."""
    L = lib()
    n = pts.shape[0]
    h = np.zeros(n)
    iters = np.zeros(n, dtype=np.int32)

    def fn(rows, d, idx):
        d = _f64(d)
        hh = np.zeros(rows.size)
        st = np.zeros(rows.size, dtype=np.int32)
        it = np.zeros(rows.size, dtype=np.int32)
        L.orc_solve_h(rows.size, d.shape[1], _p(d), eta, kappa, _p(hh), _p(st, _i32),
                      _p(it, _i32))
        if np.any(st == 2):
            raise OracleError(RT_ENOCONV, "smoothing length did not converge")
        ok = st == 0
        h[rows[ok]] = hh[ok]
        iters[rows[ok]] = it[ok]
        return ok

    blocks = _knn_covering(tree, pts, fn)
    if return_blocks:
        return h, iters, blocks
    return h, iters


def gather_lists(tree: cKDTree, x: np.ndarray, H: np.ndarray, blocks=None):
    """CSR of G(i) = {j != i : r_ij < H_i}, rows sorted by partner index.
    `blocks` are candidate rows whose last distance reaches H (reused from the
    smoothing-length solve when available)."""
    n = x.shape[0]
    if blocks is None:
        blocks = _knn_covering(tree, x, lambda rows, d, idx: d[:, -1] >= H[rows])
    counts = np.zeros(n, dtype=np.int64)
    parts = []
    big = np.iinfo(np.int64).max
    for rows, d, idx in blocks:
        if not np.all(d[:, -1] >= H[rows]):
            raise OracleError(-1, "candidate rows do not cover the compact support")
        m = (d < H[rows][:, None]) & (idx != rows[:, None])
        sel = np.where(m, idx, big)
        sel.sort(axis=1)
        c = m.sum(axis=1)
        counts[rows] = c
        parts.append((rows, sel, c))
    ptr = np.zeros(n + 1, dtype=np.int64)
    ptr[1:] = np.cumsum(counts)
    out = np.zeros(ptr[-1], dtype=np.int64)
    for rows, sel, c in parts:
        w = sel.shape[1]
        keep = np.arange(w)[None, :] < c[:, None]
        dst = ptr[rows][:, None] + np.arange(w)[None, :]
        out[dst[keep]] = sel[keep]
    return _i64a(ptr), _i64a(out)


def symmetric_lists(n: int, gptr: np.ndarray, gidx: np.ndarray):
    """CSR of N(i) = G(i) union G^T(i), rows sorted, no duplicates."""
    L = lib()
    tptr = np.zeros(n + 1, dtype=np.int64)
    tidx = np.zeros(gidx.size, dtype=np.int64)
    fill = np.zeros(n, dtype=np.int64)
    L.orc_transpose(n, _p(gptr, _i64), _p(gidx, _i64), _p(tptr, _i64), _p(tidx, _i64),
                    _p(fill, _i64))
    sptr = np.zeros(n + 1, dtype=np.int64)
    tot = L.orc_sym_count(n, _p(gptr, _i64), _p(gidx, _i64), _p(tptr, _i64),
                          _p(tidx, _i64), _p(sptr, _i64))
    sidx = np.zeros(max(tot, 1), dtype=np.int64)
    L.orc_sym_fill(n, _p(gptr, _i64), _p(gidx, _i64), _p(tptr, _i64), _p(tidx, _i64),
                   _p(sptr, _i64), _p(sidx, _i64))
    return sptr, sidx[:tot]


# ---------------------------------------------------------------------------
# static geometry

@dataclasses.dataclass
class Geometry:
    x: np.ndarray
    h: np.ndarray
    H: np.ndarray
    omega: np.ndarray
    V: np.ndarray
    E: np.ndarray        # (n, 3, 3)
    B: np.ndarray        # (n, 3, 3)
    gptr: np.ndarray
    gidx: np.ndarray
    sptr: np.ndarray
    sidx: np.ndarray
    dt: float
    box: np.ndarray
    c: float
    cfl: float
    eta: float
    kappa: float
    h_iters: Optional[np.ndarray] = None
    tree: Optional[cKDTree] = None

    @property
    def n(self):
        return self.x.shape[0]

    @property
    def n_pairs(self) -> int:
        """Unordered interacting pairs (r_kl < max(H_k, H_l))."""
        return int(self.sidx.size // 2)


def build_geometry(x, eta: float = ETA, kappa: float = KAPPA, c: float = 1.0,
                   cfl: float = 0.9, h: Optional[np.ndarray] = None,
                   box: float = 1.0) -> Geometry:
    L = lib()
    x = _f64(x)
    n = x.shape[0]
    boxv = np.full(3, float(box))
    tree = cKDTree(x, boxsize=box)
    iters, blocks = None, None
    if h is None:
        h, iters, blocks = solve_h(tree, x, eta, kappa, return_blocks=True)
    h = _f64(h)
    H = kappa * h
    if np.any(H >= 0.5 * box):
        raise OracleError(-1, "compact support exceeds half the box")
    gptr, gidx = gather_lists(tree, x, H, blocks)
    sptr, sidx = symmetric_lists(n, gptr, gidx)
    omega = np.zeros(n)
    V = np.zeros(n)
    E = np.zeros((n, 9))
    L.orc_geometry(n, _p(x), _p(H), _p(boxv), _p(gptr, _i64), _p(gidx, _i64),
                   _p(omega), _p(V), _p(E))
    E = E.reshape(n, 3, 3)
    ev = np.linalg.eigvalsh(E)
    if np.any(ev[:, 0] <= 1e-12 * np.maximum(ev[:, 2], 1e-300)):
        raise OracleError(RT_ESINGULAR, "singular E matrix (coplanar neighbourhood)")
    B = np.linalg.inv(E)
    dt = L.orc_dt(n, _p(V), cfl, c)
    return Geometry(x, h, H, omega, V, E, _f64(B), gptr, gidx, sptr, sidx, dt, boxv,
                    c, cfl, eta, kappa, iters, tree)


@dataclasses.dataclass
class Sources:
    xs: np.ndarray
    h: np.ndarray
    src: np.ndarray     # entry -> source
    gas: np.ndarray     # entry -> gas particle
    xi: np.ndarray      # entry weight xi_sg
    qnz: np.ndarray


def build_sources(geom: Geometry, xs, eta_star: float = ETA) -> Sources:
    L = lib()
    xs = _f64(xs).reshape(-1, 3)
    S = xs.shape[0]
    if S == 0:
        z = np.zeros(0, np.int64)
        return Sources(xs, np.zeros(0), z, z, np.zeros(0), np.zeros(0, np.int32))
    hs, _, blocks = solve_h(geom.tree, xs, eta_star, geom.kappa, return_blocks=True)
    Hs = geom.kappa * hs
    src, gas, xi, qnz = [], [], [], []
    cand = {}
    for rows, d, idx in blocks:
        for r_, dd, ii in zip(rows, d, idx):
            cand[int(r_)] = ii[dd < Hs[r_]]
    for s in range(S):
        g = np.sort(cand[s])
        xg = _f64(geom.x[g])
        wts = np.zeros(g.size)
        q = L.orc_source_weights(g.size, _p(_f64(xs[s])), _p(xg), Hs[s], _p(geom.box),
                                 _p(wts))
        if q < 0:
            raise OracleError(-1, "source without gas neighbours")
        src.append(np.full(g.size, s, np.int64))
        gas.append(g)
        xi.append(wts)
        qnz.append(q)
    src, gas, xi = np.concatenate(src), np.concatenate(gas), np.concatenate(xi)
    order = np.lexsort((src, gas))
    return Sources(xs, hs, _i64a(src[order]), _i64a(gas[order]), _f64(xi[order]),
                   np.asarray(qnz, np.int32))


# ---------------------------------------------------------------------------
# per-step operators

def inject(geom: Geometry, srcs: Sources, U: np.ndarray, L: np.ndarray,
           dt: Optional[float] = None) -> None:
    """In place: E_g += dt * sum_s xi_sg L_s / V_g."""
    if srcs is None or srcs.src.size == 0:
        return
    dt = geom.dt if dt is None else dt
    assert U.flags.c_contiguous and U.dtype == np.float64
    Lm = _f64(L)
    lib().orc_inject(srcs.src.size, U.shape[1], _p(srcs.src, _i64), _p(srcs.gas, _i64),
                     _p(srcs.xi), _p(geom.V), _p(Lm), dt, _p(U))


def gradient(geom: Geometry, U: np.ndarray) -> np.ndarray:
    U = _f64(U)
    n, G = U.shape[0], U.shape[1]
    dU = np.zeros((n, G, 4, 3))
    lib().orc_gradient(n, G, _p(geom.x), _p(geom.H), _p(geom.V), _p(_f64(geom.B)),
                       _p(geom.box), _p(geom.gptr, _i64), _p(geom.gidx, _i64), _p(U),
                       _p(dU))
    return dU


def ivanova_sums(geom: Geometry) -> np.ndarray:
    """[n][3]: sum_k grad W_k(x_i) over the gather neighbours of each particle
    (the normalisation-gradient term of the Ivanova surfaces)."""
    g = np.zeros((geom.n, 3))
    lib().orc_ivanova_sums(geom.n, _p(geom.x), _p(geom.H), _p(geom.box),
                           _p(geom.gptr, _i64), _p(geom.gidx, _i64), _p(g))
    return g


def grad_psi(geom: Geometry, gsum: np.ndarray, i: int, j: int) -> np.ndarray:
    """grad psi_j(x_i) of the Ivanova surfaces (analytic, H_i held fixed)."""
    out = np.zeros(3)
    lib().orc_grad_psi(_p(_f64(geom.x[i])), _p(_f64(geom.x[j])), geom.H[i], geom.V[i],
                       _p(_f64(gsum[i])), _p(geom.box), _p(out))
    return out


def surface_ivanova(geom: Geometry, gsum: np.ndarray, k: int, l: int) -> np.ndarray:
    A = np.zeros(3)
    lib().orc_surface_ivanova(_p(_f64(geom.x[k])), _p(_f64(geom.x[l])), geom.H[k], geom.H[l],
                              geom.V[k], geom.V[l], _p(_f64(gsum[k])), _p(_f64(gsum[l])),
                              _p(geom.box), _p(A))
    return A


def transport(geom: Geometry, U: np.ndarray, dU: np.ndarray, dt: Optional[float] = None,
              hll: Optional[np.ndarray] = None, ivanova: bool = False):
    """Returns (U_new, counts[4], ledger[G]).  hll: an eigenvalue table
    (hll_table()) selects the HLL solver instead of GLF; ivanova: the Ivanova
    surfaces (eq:IvanovaAij) instead of the Hopkins ones."""
    U, dU = _f64(U), _f64(dU)
    n, G = U.shape[0], U.shape[1]
    dt = geom.dt if dt is None else dt
    out = np.zeros_like(U)
    counts = np.zeros(4, dtype=np.int64)
    ledger = np.zeros(G)
    args = (n, G, _p(geom.x), _p(geom.h), _p(geom.H), _p(geom.V), _p(_f64(geom.B)),
            _p(geom.box), _p(geom.sptr, _i64), _p(geom.sidx, _i64), geom.c, dt, _p(U), _p(dU),
            _p(out), _p(counts, _i64), _p(ledger))
    if ivanova:
        gsum = ivanova_sums(geom)
        tab = None if hll is None else _f64(hll)
        lib().orc_transport_ivanova(*args, None if tab is None else _p(tab),
                                    0 if tab is None else tab.shape[0],
                                    0 if tab is None else tab.shape[1], _p(gsum))
    elif hll is None:
        lib().orc_transport(*args)
    else:
        tab = _f64(hll)
        lib().orc_transport_hll(*args, _p(tab), tab.shape[0], tab.shape[1])
    return out, counts, ledger


# HLL solver (eq:riemann-HLL): extreme eigenvalues of the M1 flux Jacobian

def m1_flux_printed(U: np.ndarray, n: np.ndarray, c: float = 1.0) -> np.ndarray:
    """(F.n, c^2 P n) of one state with the closure as printed
    (eq:eddington-group), in any dtype (complex steps included)."""
    E, F = U[0], U[1:]
    Fn = np.sqrt(F @ F)
    f = Fn / (c * E)
    chi = (3 + 4 * f * f) / (5 + 2 * np.sqrt(4 - 3 * f * f))
    nf = F / Fn
    D = (1 - chi) / 2 * np.eye(3) + (3 * chi - 1) / 2 * np.outer(nf, nf)
    return np.concatenate([[F @ n], c * c * E * (D @ n)])


def m1_jacobian(f: float, mu: float, c: float = 1.0) -> np.ndarray:
    """d(F.n, c^2 P n)/d(E, F) at E = 1, F = c f e_x, n = (mu, sqrt(1-mu^2), 0),
    by complex steps (exact to rounding), for 0 < f < 1."""
    n = np.array([mu, np.sqrt(max(0.0, 1.0 - mu * mu)), 0.0])
    U = np.array([1.0, c * f, 0.0, 0.0])
    J = np.zeros((4, 4))
    hstep = 1e-30
    for k in range(4):
        Uc = U.astype(complex)
        Uc[k] += 1j * hstep
        J[:, k] = m1_flux_printed(Uc, n, c).imag / hstep
    return J


def hll_table(nf: int = 65, nmu: int = 65) -> np.ndarray:
    """[nf][nmu][2] = (l_min, l_max) / c at f = i/(nf-1), mu = -1 + 2 j/(nmu-1):
    the extreme eigenvalues of m1_jacobian (numpy's general eigensolver); at
    f = 0 they are -+1/sqrt(3) for every mu, at f = 1 all four eigenvalues are
    mu (the free-streaming limit)."""
    tab = np.zeros((nf, nmu, 2))
    for i in range(nf):
        f = i / (nf - 1)
        for j in range(nmu):
            mu = -1.0 + 2.0 * j / (nmu - 1)
            if i == 0:
                tab[i, j] = (-1.0 / np.sqrt(3.0), 1.0 / np.sqrt(3.0))
            elif i == nf - 1:
                tab[i, j] = (mu, mu)
            else:
                ev = np.linalg.eigvals(m1_jacobian(f, mu)).real
                tab[i, j] = (ev.min(), ev.max())
    return tab


def hll_flux(qL, qR, nh, tab, c: float = 1.0) -> np.ndarray:
    phi = np.zeros(4)
    t = _f64(tab)
    lib().orc_hll(_p(_f64(qL)), _p(_f64(qR)), _p(_f64(nh)), c, _p(t), t.shape[0], t.shape[1],
                  _p(phi))
    return phi


def photon_total(geom: Geometry, U: np.ndarray) -> np.ndarray:
    U = _f64(U)
    Q = np.zeros(U.shape[1])
    lib().orc_photon_total(U.shape[0], U.shape[1], _p(geom.V), _p(U), _p(Q))
    return Q


def drift(geom: Geometry, U: np.ndarray, dx: np.ndarray, dU: Optional[np.ndarray] = None):
    """Drift correction (rt_oracle.c orc_drift): U extrapolated by the
    displacements dx [n][3] with its gradients (computed when dU is None).
    Returns (U_new, counts[4], ledger[G])."""
    U = _f64(U)
    dU = gradient(geom, U) if dU is None else _f64(dU)
    dx = _f64(dx)
    n, G = U.shape[:2]
    out = np.empty_like(U)
    counts = np.zeros(4, dtype=np.int64)
    ledger = np.zeros(G)
    lib().orc_drift(n, G, _p(U), _p(dU), _p(dx), _p(geom.V), geom.c, _p(out),
                    _p(counts, _i64), _p(ledger))
    return out, counts, ledger


def absorb(geom: Geometry, U: np.ndarray, n_old: np.ndarray, sigma: np.ndarray, dt: float,
           n_new: Optional[np.ndarray] = None, c: Optional[float] = None):
    """Photon removal of the thermochemistry step (rt_oracle.c orc_absorb).
    n_old, n_new [n][J] species densities, sigma [G][J].  Returns (U_new,
    absorbed[G])."""
    U = _f64(U)
    n_old = _f64(n_old)
    sigma = _f64(sigma)
    G, J = sigma.shape
    out = np.empty_like(U)
    absorbed = np.zeros(G)
    nn = None if n_new is None else _f64(n_new)
    lib().orc_absorb(U.shape[0], G, J, _p(geom.V), _p(U), _p(n_old),
                     None if nn is None else _p(nn), _p(sigma),
                     geom.c if c is None else c, dt, _p(out), _p(absorbed))
    return out, absorbed


def surface(geom: Geometry, k: int, l: int) -> np.ndarray:
    A = np.zeros(3)
    B = _f64(geom.B)
    lib().orc_surface(_p(_f64(geom.x[k])), _p(_f64(geom.x[l])), geom.H[k], geom.H[l],
                      geom.V[k], geom.V[l], _p(_f64(B[k])), _p(_f64(B[l])), _p(geom.box),
                      _p(A))
    return A


def step(geom: Geometry, srcs: Optional[Sources], U: np.ndarray, L=None,
         dt: Optional[float] = None, hll: Optional[np.ndarray] = None,
         ivanova: bool = False):
    """One RT step in the operator-splitting order inject -> gradient ->
    transport.  Returns (U_new, info)."""
    U = _f64(U).copy()
    if srcs is not None and srcs.src.size:
        inject(geom, srcs, U, L, dt)
    dU = gradient(geom, U)
    out, counts, ledger = transport(geom, U, dU, dt, hll=hll, ivanova=ivanova)
    return out, {"counts": counts, "ledger": ledger, "U_injected": U, "dU": dU}


def run(geom: Geometry, srcs: Optional[Sources], U0: np.ndarray, L, steps: int,
        keep: bool = False, hll: Optional[np.ndarray] = None, ivanova: bool = False):
    U = _f64(U0).copy()
    counts = np.zeros(4, dtype=np.int64)
    ledger = np.zeros(U.shape[1])
    states = [U.copy()] if keep else None
    for _ in range(steps):
        U, info = step(geom, srcs, U, L, hll=hll, ivanova=ivanova)
        counts += info["counts"]
        ledger += info["ledger"]
        if keep:
            states.append(U.copy())
    return U, {"counts": counts, "ledger": ledger, "states": states}


# individual time steps (Part II "Individual time steps", Part III
# eq:transport-update-explicit with min{dt_k, dt_l}, factor-4 limiter)

def time_bins(geom: Geometry, nmax: int) -> np.ndarray:
    """b_i: dt_i = dt_min 2^b_i, the largest n <= nmax with dt_min 2^n within
    particle i's own CFL step, lowered to |b_k - b_l| <= 2 for interacting
    pairs.  dt_min = geom.dt (the smallest CFL step)."""
    b = np.zeros(geom.n, dtype=np.int32)
    lib().orc_bins(geom.n, _p(geom.V), geom.cfl, geom.c, geom.dt, int(nmax),
                   _p(geom.sptr, _i64), _p(geom.sidx, _i64), _p(b, _i32))
    return b


def active(bins: np.ndarray, tick: int) -> np.ndarray:
    """Particles that end a step at the end of tick `tick`."""
    return ((tick + 1) % (np.int64(1) << bins.astype(np.int64))) == 0


def run_binned(geom: Geometry, srcs: Optional[Sources], U0: np.ndarray, L, ticks: int,
               bins: np.ndarray, t0: int = 0, dU=None, acc=None,
               hll: Optional[np.ndarray] = None, ivanova: bool = False):
    """`ticks` ticks of the individual-time-step scheme from tick t0.  Every
    particle starts with the gradient of U0 (unless dU is given); in tick t the
    particles that end a step inject (with their own dt), recompute their
    gradient, and apply their flux sums, while every pair whose smaller bin ends
    a step exchanges dt_kl |A| Phi (GLF, or HLL with the table `hll`; the
    Hopkins surfaces, or the Ivanova ones with `ivanova`).
    Returns (U, info) with info["acc"] (the pending flux sums) and info["dU"]
    (the stored gradients)."""
    U = _f64(U0).copy()
    n, G = U.shape[0], U.shape[1]
    bins = np.ascontiguousarray(bins, dtype=np.int32)
    dU = gradient(geom, U) if dU is None else _f64(dU).copy()
    acc = np.zeros_like(U) if acc is None else _f64(acc).copy()
    counts = np.zeros(4, dtype=np.int64)
    ledger = np.zeros(G)
    Lm = _f64(L) if (srcs is not None and srcs.src.size) else None
    tab = None if hll is None else _f64(hll)
    gsum = ivanova_sums(geom) if ivanova else None
    for t in range(t0, t0 + ticks):
        act = active(bins, t)
        if Lm is not None:
            lib().orc_inject_binned(srcs.src.size, G, _p(srcs.src, _i64), _p(srcs.gas, _i64),
                                    _p(srcs.xi), _p(geom.V), _p(Lm), geom.dt, _p(bins, _i32),
                                    t, _p(U))
        if act.any():
            dU[act] = gradient(geom, U)[act]
        out = np.zeros_like(U)
        lib().orc_transport_binned(n, G, _p(geom.x), _p(geom.h), _p(geom.H), _p(geom.V),
                                   _p(_f64(geom.B)), _p(geom.box), _p(geom.sptr, _i64),
                                   _p(geom.sidx, _i64), geom.c, geom.dt, _p(bins, _i32), t,
                                   _p(U), _p(dU), _p(acc), _p(out), _p(counts, _i64),
                                   _p(ledger), None if tab is None else _p(tab),
                                   0 if tab is None else tab.shape[0],
                                   0 if tab is None else tab.shape[1],
                                   None if gsum is None else _p(gsum))
        U = out
    return U, {"acc": acc, "dU": dU, "counts": counts, "ledger": ledger}


def num_threads() -> int:
    return int(lib().orc_num_threads())


def set_num_threads(t: int) -> None:
    """Threads of the C oracle's parallel loops (results do not depend on it)."""
    lib().orc_set_num_threads(int(t))
