"""Python binding of the gfx950 photon-transport library (libgearrt.so).

Argument marshalling only: every array lives in device memory as a torch
tensor, the calls below pass raw device pointers and torch's current HIP
stream to the C ABI declared in include/rt.h, and every step of the transport
runs in the library's HIP kernels.  There is no CPU fallback: importing this
module without the built library raises.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgearrt.so")

RT_OK, RT_EINVAL, RT_ENOMEM, RT_EHIP, RT_ENOCONV, RT_ESINGULAR, RT_ESTATE = 0, -1, -2, -3, -4, -5, -6
RT_ENONFINITE = -7
RT_FP64, RT_FP32C = 0, 1
RT_GLF, RT_HLL = 0, 1
RT_HOPKINS, RT_IVANOVA = 0, 1
RT_HLL_NF, RT_HLL_NMU = 65, 65
STATUS_NAMES = {0: "RT_OK", -1: "RT_EINVAL", -2: "RT_ENOMEM", -3: "RT_EHIP",
                -4: "RT_ENOCONV", -5: "RT_ESINGULAR", -6: "RT_ESTATE", -7: "RT_ENONFINITE"}

KAPPA = 1.825742
ETA = 1.2348

EXPORTED = ["rt_create", "rt_destroy", "rt_last_error", "rt_set_stream", "rt_build_cells",
            "rt_set_sources", "rt_inject", "rt_gradient", "rt_transport", "rt_photon_total",
            "rt_adjoint", "rt_sync", "rt_get_stats", "rt_get_geometry", "rt_get_neighbours",
            "rt_get_sources", "rt_timing", "rt_get_timing", "rt_time_bins", "rt_tick",
            "rt_set_riemann", "rt_get_hll_table", "rt_photon_groups", "rt_absorb", "rt_drift",
            "rt_set_surfaces", "rt_set_h_iterations", "rt_adjoint_static"]


class RTError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


class rt_params(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("groups", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("box", ctypes.c_double), ("eta", ctypes.c_double), ("kappa", ctypes.c_double),
                ("c_red", ctypes.c_double), ("cfl", ctypes.c_double),
                ("hip_stream", ctypes.c_void_p)]


class rt_stats(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("n_entries", ctypes.c_int64), ("n_pairs", ctypes.c_int64),
                ("n_gather", ctypes.c_int64), ("sell_slots", ctypes.c_int64),
                ("max_neighbours", ctypes.c_int32), ("h_iter_max", ctypes.c_int32),
                ("n_inject", ctypes.c_int64), ("device_bytes", ctypes.c_int64),
                ("device_bytes_peak", ctypes.c_int64), ("h_list_overflow", ctypes.c_int64),
                ("union_blocks", ctypes.c_int64), ("union_staged_blocks", ctypes.c_int64),
                ("adj_union_blocks", ctypes.c_int64), ("adj_union_staged_blocks", ctypes.c_int64),
                ("task_longest", ctypes.c_int64), ("task_bound", ctypes.c_int64)]


_lib = None
_VP = ctypes.c_void_p


def load_library() -> ctypes.CDLL:
    """Load libgearrt.so (built by __graft_entry__.build()); raise if absent.
    GEARRT_LIB names another build of the same library (for example one with
    different tuning macros, see build.build(defines=...))."""
    global _lib
    if _lib is not None:
        return _lib
    path = os.environ.get("GEARRT_LIB", LIB_PATH)
    if not os.path.exists(path):
        raise ImportError(f"HIP library {path} is not built; run __graft_entry__.build()")
    L = ctypes.CDLL(path)
    i32 = ctypes.c_int32
    L.rt_create.argtypes = [ctypes.POINTER(rt_params), ctypes.POINTER(_VP)]
    L.rt_destroy.argtypes = [_VP]
    L.rt_destroy.restype = None
    L.rt_last_error.argtypes = [_VP]
    L.rt_last_error.restype = ctypes.c_char_p
    L.rt_set_stream.argtypes = [_VP, _VP]
    L.rt_build_cells.argtypes = [_VP] * 7
    L.rt_set_sources.argtypes = [_VP, i32, _VP, ctypes.c_double]
    L.rt_set_h_iterations.argtypes = [_VP, i32]
    L.rt_inject.argtypes = [_VP] * 4
    L.rt_gradient.argtypes = [_VP] * 3
    L.rt_transport.argtypes = [_VP] * 8
    L.rt_photon_total.argtypes = [_VP] * 3
    L.rt_adjoint.argtypes = [_VP] * 9
    L.rt_adjoint_static.argtypes = [_VP] * 8
    L.rt_time_bins.argtypes = [_VP, i32, _VP, ctypes.POINTER(ctypes.c_int64)]
    L.rt_tick.argtypes = [_VP, _VP, _VP, ctypes.c_int64, _VP, _VP, _VP, _VP, _VP]
    L.rt_photon_groups.argtypes = [i32, _VP, ctypes.c_double, _VP, _VP, _VP, _VP]
    L.rt_absorb.argtypes = [_VP, _VP, i32, _VP, _VP, _VP, _VP, _VP, _VP]
    L.rt_drift.argtypes = [_VP] * 7
    L.rt_set_riemann.argtypes = [_VP, i32]
    L.rt_set_surfaces.argtypes = [_VP, i32]
    L.rt_get_hll_table.argtypes = [_VP, _VP]
    L.rt_sync.argtypes = [_VP]
    L.rt_get_stats.argtypes = [_VP, ctypes.POINTER(rt_stats)]
    L.rt_get_geometry.argtypes = [_VP] * 4
    L.rt_get_neighbours.argtypes = [_VP] * 3
    L.rt_get_sources.argtypes = [_VP] * 5
    L.rt_timing.argtypes = [_VP, i32]
    L.rt_get_timing.argtypes = [_VP, ctypes.c_char_p, ctypes.POINTER(ctypes.c_double),
                                ctypes.POINTER(ctypes.c_int64)]
    _lib = L
    return L


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _need(t: torch.Tensor, name: str, dtype, shape=None):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must live in device memory")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")


def hll_speed_table() -> np.ndarray:
    """The library's HLL wave-speed table, [RT_HLL_NF][RT_HLL_NMU][2]
    (l_min, l_max) in units of c, as a host float64 array (host code only)."""
    L = load_library()
    tab = np.zeros((RT_HLL_NF, RT_HLL_NMU, 2), dtype=np.float64)
    st = L.rt_get_hll_table(None, ctypes.c_void_p(tab.ctypes.data))
    if st != RT_OK:
        raise RTError(st, L.rt_last_error(None).decode())
    return tab


def photon_groups(edges_eV, T_bb: float):
    """Group constants of the library (host code): returns (sigma_N [G][3],
    sigma_E [G][3] in cm^2 for H0, He0, He+; eps [G] in erg; frac [G])."""
    L = load_library()
    e = np.ascontiguousarray(edges_eV, dtype=np.float64)
    G = e.size - 1
    sN, sE = np.zeros((G, 3)), np.zeros((G, 3))
    eps, frac = np.zeros(G), np.zeros(G)
    vp = lambda a: ctypes.c_void_p(a.ctypes.data)
    st = L.rt_photon_groups(G, vp(e), float(T_bb), vp(sN), vp(sE), vp(eps), vp(frac))
    if st != RT_OK:
        raise RTError(st, L.rt_last_error(None).decode())
    return sN, sE, eps, frac


class RT:
    """One library context (rt_ctx) for a static particle set."""

    def __init__(self, n: int, groups: int, precision: str = "fp64", box: float = 1.0,
                 eta: float = ETA, kappa: float = KAPPA, c_red: float = 1.0, cfl: float = 0.9,
                 device: Optional[torch.device] = None):
        self.L = load_library()
        self.n, self.G = int(n), int(groups)
        self.precision = precision
        self.sdtype = torch.float64 if precision == "fp64" else torch.float32
        self.device = torch.device("cuda") if device is None else torch.device(device)
        stream = torch.cuda.current_stream(self.device).cuda_stream
        self.params = rt_params(self.n, self.G, RT_FP64 if precision == "fp64" else RT_FP32C,
                                box, eta, kappa, c_red, cfl, stream)
        h = _VP()
        st = self.L.rt_create(ctypes.byref(self.params), ctypes.byref(h))
        if st != RT_OK:
            raise RTError(st, self.L.rt_last_error(None).decode())
        self.ctx = h
        self.S = 0
        self.dt = None
        self.perm = None

    def __del__(self):
        try:
            if getattr(self, "ctx", None):
                self.L.rt_destroy(self.ctx)
                self.ctx = None
        except Exception:
            pass

    # -- plumbing -----------------------------------------------------------
    def _check(self, st: int):
        if st != RT_OK:
            raise RTError(st, self.L.rt_last_error(self.ctx).decode())

    def _bind_stream(self):
        self.L.rt_set_stream(self.ctx, ctypes.c_void_p(torch.cuda.current_stream(self.device).cuda_stream))

    def state(self, fill: float = 0.0) -> torch.Tensor:
        return torch.full((self.n, self.G, 4), fill, dtype=self.sdtype, device=self.device)

    def grad_buffer(self) -> torch.Tensor:
        """Gradient record UD [n, G, 16]: per group the state (4) then its
        gradients (4 x 3)."""
        return torch.empty((self.n, self.G, 16), dtype=self.sdtype, device=self.device)

    def gradients_of(self, UD: torch.Tensor) -> torch.Tensor:
        """The gradient part of UD as [n, G, 4, 3]."""
        return UD[:, :, 4:].reshape(self.n, self.G, 4, 3)

    def states_of(self, UD: torch.Tensor) -> torch.Tensor:
        """The state part of UD as [n, G, 4]."""
        return UD[:, :, :4]

    # -- the C entry points ---------------------------------------------------
    def rt_build_cells(self, x: torch.Tensor, h_in: Optional[torch.Tensor] = None):
        """Returns (perm, h, V, dt): Morton permutation and sorted-order h, V,
        and the global time step (device scalar)."""
        _need(x, "x", torch.float64, (self.n, 3))
        if h_in is not None:
            _need(h_in, "h_in", torch.float64, (self.n,))
        perm = torch.empty(self.n, dtype=torch.int64, device=self.device)
        h = torch.empty(self.n, dtype=torch.float64, device=self.device)
        V = torch.empty(self.n, dtype=torch.float64, device=self.device)
        dt = torch.empty(1, dtype=torch.float64, device=self.device)
        self._bind_stream()
        self._check(self.L.rt_build_cells(self.ctx, _ptr(x), _ptr(h_in), _ptr(perm), _ptr(h),
                                          _ptr(V), _ptr(dt)))
        self.perm, self.h, self.V, self.dt = perm, h, V, dt
        return perm, h, V, dt

    def rt_set_sources(self, xs: torch.Tensor, eta_star: float = ETA):
        S = 0 if xs is None else int(xs.shape[0])
        if S:
            _need(xs, "xs", torch.float64, (S, 3))
        self._bind_stream()
        self._check(self.L.rt_set_sources(self.ctx, S, _ptr(xs) if S else None, eta_star))
        self.S = S

    def rt_inject(self, U: torch.Tensor, L: torch.Tensor, dt: Optional[torch.Tensor] = None):
        _need(U, "U", self.sdtype, (self.n, self.G, 4))
        _need(L, "L", torch.float64, (self.S, self.G))
        dt = self.dt if dt is None else dt
        self._bind_stream()
        self._check(self.L.rt_inject(self.ctx, _ptr(U), _ptr(L), _ptr(dt)))

    def rt_absorb(self, U: torch.Tensor, n_old: torch.Tensor, sigma: torch.Tensor,
                  n_new: Optional[torch.Tensor] = None, dt: Optional[torch.Tensor] = None,
                  photon_total: Optional[torch.Tensor] = None,
                  absorbed: Optional[torch.Tensor] = None) -> torch.Tensor:
        """Photon removal of the thermochemistry step, in place on U."""
        _need(U, "U", self.sdtype, (self.n, self.G, 4))
        _need(sigma, "sigma", torch.float64)
        if sigma.dim() != 2 or sigma.shape[0] != self.G:
            raise ValueError(f"sigma must have shape ({self.G}, J)")
        J = int(sigma.shape[1])
        _need(n_old, "n_old", torch.float64, (self.n, J))
        if n_new is not None:
            _need(n_new, "n_new", torch.float64, (self.n, J))
        if photon_total is not None:
            _need(photon_total, "photon_total", torch.float64, (self.G,))
        if absorbed is not None:
            _need(absorbed, "absorbed", torch.float64, (self.G,))
        dt = self.dt if dt is None else dt
        self._bind_stream()
        self._check(self.L.rt_absorb(self.ctx, _ptr(U), J, _ptr(n_old), _ptr(n_new),
                                     _ptr(sigma), _ptr(dt), _ptr(photon_total), _ptr(absorbed)))
        return U

    def rt_drift(self, UD: torch.Tensor, dx: torch.Tensor, U_out: Optional[torch.Tensor] = None,
                 photon_total: Optional[torch.Tensor] = None,
                 counts: Optional[torch.Tensor] = None,
                 ledger: Optional[torch.Tensor] = None) -> torch.Tensor:
        """Drift correction: the states of UD extrapolated by the displacements dx."""
        _need(UD, "UD", self.sdtype, (self.n, self.G, 16))
        _need(dx, "dx", torch.float64, (self.n, 3))
        U_out = torch.empty((self.n, self.G, 4), dtype=self.sdtype, device=self.device) \
            if U_out is None else U_out
        _need(U_out, "U_out", self.sdtype, (self.n, self.G, 4))
        if photon_total is not None:
            _need(photon_total, "photon_total", torch.float64, (self.G,))
        if counts is not None:
            _need(counts, "counts", torch.int64, (4,))
        if ledger is not None:
            _need(ledger, "ledger", torch.float64, (self.G,))
        self._bind_stream()
        self._check(self.L.rt_drift(self.ctx, _ptr(UD), _ptr(dx), _ptr(U_out), _ptr(photon_total),
                                    _ptr(counts), _ptr(ledger)))
        return U_out

    def rt_gradient(self, U: torch.Tensor, UD: Optional[torch.Tensor] = None) -> torch.Tensor:
        _need(U, "U", self.sdtype, (self.n, self.G, 4))
        UD = self.grad_buffer() if UD is None else UD
        _need(UD, "UD", self.sdtype, (self.n, self.G, 16))
        self._bind_stream()
        self._check(self.L.rt_gradient(self.ctx, _ptr(U), _ptr(UD)))
        return UD

    def rt_transport(self, UD, dt=None, U_out=None, photon_total=None, counts=None,
                     ledger=None, U_unguarded=None) -> torch.Tensor:
        _need(UD, "UD", self.sdtype, (self.n, self.G, 16))
        dt = self.dt if dt is None else dt
        _need(dt, "dt", torch.float64, (1,))
        if U_out is None:
            U_out = torch.empty((self.n, self.G, 4), dtype=self.sdtype, device=self.device)
        _need(U_out, "U_out", self.sdtype, (self.n, self.G, 4))
        if photon_total is not None:
            _need(photon_total, "photon_total", torch.float64, (self.G,))
        if counts is not None:
            _need(counts, "counts", torch.int64, (4,))
        if ledger is not None:
            _need(ledger, "ledger", torch.float64, (self.G,))
        if U_unguarded is not None:
            _need(U_unguarded, "U_unguarded", self.sdtype, (self.n, self.G, 4))
        self._bind_stream()
        self._check(self.L.rt_transport(self.ctx, _ptr(UD), _ptr(dt), _ptr(U_out),
                                        _ptr(photon_total), _ptr(counts), _ptr(ledger),
                                        _ptr(U_unguarded)))
        return U_out

    def rt_time_bins(self, max_bin: int, bins: Optional[torch.Tensor] = None):
        """Individual time bins (dt_i = dt 2^b_i, limited to 2 bins between
        interacting particles).  Returns (bins [n] int32, ticks per full cycle)."""
        if bins is None:
            bins = torch.empty(self.n, dtype=torch.int32, device=self.device)
        _need(bins, "bins", torch.int32, (self.n,))
        cyc = ctypes.c_int64(0)
        self._bind_stream()
        self._check(self.L.rt_time_bins(self.ctx, int(max_bin), _ptr(bins), ctypes.byref(cyc)))
        return bins, int(cyc.value)

    def rt_tick(self, U, L, tick: int, UD, acc, photon_total=None, counts=None, ledger=None):
        """One tick of the individual-time-step scheme (U, UD, acc in/out)."""
        _need(U, "U", self.sdtype, (self.n, self.G, 4))
        _need(UD, "UD", self.sdtype, (self.n, self.G, 16))
        _need(acc, "acc", torch.float64, (self.n, self.G, 4))
        if L is not None:
            _need(L, "L", torch.float64, (self.S, self.G))
        if photon_total is not None:
            _need(photon_total, "photon_total", torch.float64, (self.G,))
        if counts is not None:
            _need(counts, "counts", torch.int64, (4,))
        if ledger is not None:
            _need(ledger, "ledger", torch.float64, (self.G,))
        self._bind_stream()
        self._check(self.L.rt_tick(self.ctx, _ptr(U), _ptr(L), int(tick), _ptr(UD), _ptr(acc),
                                   _ptr(photon_total), _ptr(counts), _ptr(ledger)))
        return U

    def rt_set_h_iterations(self, max_iter: int):
        """Iteration cap of the smoothing-length solve of later builds."""
        self._check(self.L.rt_set_h_iterations(self.ctx, int(max_iter)))

    def rt_set_riemann(self, solver: str):
        """Riemann solver of rt_transport: "glf" or "hll"."""
        code = {"glf": RT_GLF, "hll": RT_HLL}[solver]
        self._check(self.L.rt_set_riemann(self.ctx, code))

    def rt_set_surfaces(self, kind: str):
        """Effective surfaces of rt_transport: "hopkins" or "ivanova"."""
        code = {"hopkins": RT_HOPKINS, "ivanova": RT_IVANOVA}[kind]
        self._bind_stream()
        self._check(self.L.rt_set_surfaces(self.ctx, code))

    def rt_get_hll_table(self):
        """The library's HLL wave-speed table (see hll_speed_table)."""
        return hll_speed_table()

    def rt_photon_total(self, U: torch.Tensor) -> torch.Tensor:
        _need(U, "U", self.sdtype, (self.n, self.G, 4))
        Q = torch.empty(self.G, dtype=torch.float64, device=self.device)
        self._bind_stream()
        self._check(self.L.rt_photon_total(self.ctx, _ptr(U), _ptr(Q)))
        return Q

    def rt_adjoint(self, U_pre, L, lam_next, lam=None, UD=None, U_unguarded=None, dL_dL=None,
                   dt=None) -> torch.Tensor:
        if U_pre is not None:
            _need(U_pre, "U_pre", self.sdtype, (self.n, self.G, 4))
        _need(lam_next, "lam_next", self.sdtype, (self.n, self.G, 4))
        lam = torch.empty_like(lam_next) if lam is None else lam
        _need(lam, "lam", self.sdtype, (self.n, self.G, 4))
        if self.S:
            _need(L, "L", torch.float64, (self.S, self.G))
        if UD is not None:
            _need(UD, "UD", self.sdtype, (self.n, self.G, 16))
        if U_unguarded is not None:
            _need(U_unguarded, "U_unguarded", self.sdtype, (self.n, self.G, 4))
        if dL_dL is not None:
            _need(dL_dL, "dL_dL", torch.float64, (self.S, self.G))
        dt = self.dt if dt is None else dt
        self._bind_stream()
        self._check(self.L.rt_adjoint(self.ctx, _ptr(U_pre), _ptr(L) if self.S else None,
                                      _ptr(dt), _ptr(UD), _ptr(U_unguarded), _ptr(lam_next),
                                      _ptr(lam), _ptr(dL_dL)))
        return lam

    def rt_adjoint_static(self, L, lam_next, UD, U_unguarded, lam=None, dL_dL=None,
                          dt=None) -> torch.Tensor:
        """rt_adjoint through the library's fixed scratch (no device
        allocation by the library); UD and U_unguarded are required."""
        _need(lam_next, "lam_next", self.sdtype, (self.n, self.G, 4))
        lam = torch.empty_like(lam_next) if lam is None else lam
        _need(lam, "lam", self.sdtype, (self.n, self.G, 4))
        _need(UD, "UD", self.sdtype, (self.n, self.G, 16))
        _need(U_unguarded, "U_unguarded", self.sdtype, (self.n, self.G, 4))
        if self.S:
            _need(L, "L", torch.float64, (self.S, self.G))
        if dL_dL is not None:
            _need(dL_dL, "dL_dL", torch.float64, (self.S, self.G))
        dt = self.dt if dt is None else dt
        self._bind_stream()
        self._check(self.L.rt_adjoint_static(self.ctx, _ptr(L) if self.S else None, _ptr(dt),
                                             _ptr(UD), _ptr(U_unguarded), _ptr(lam_next),
                                             _ptr(lam), _ptr(dL_dL)))
        return lam

    def rt_sync(self):
        self._check(self.L.rt_sync(self.ctx))

    # -- queries --------------------------------------------------------------
    def rt_get_stats(self) -> dict:
        s = rt_stats()
        self._check(self.L.rt_get_stats(self.ctx, ctypes.byref(s)))
        return {k: getattr(s, k) for k, _ in rt_stats._fields_}

    def rt_get_geometry(self):
        B = torch.empty((self.n, 6), dtype=torch.float64, device=self.device)
        nn = torch.empty(self.n, dtype=torch.int32, device=self.device)
        ng = torch.empty(self.n, dtype=torch.int32, device=self.device)
        self._check(self.L.rt_get_geometry(self.ctx, _ptr(B), _ptr(nn), _ptr(ng)))
        return B, nn, ng

    def rt_get_neighbours(self):
        st = self.rt_get_stats()
        ptr = torch.empty(self.n + 1, dtype=torch.int64, device=self.device)
        idx = torch.empty(max(st["n_entries"], 1), dtype=torch.int32, device=self.device)
        self._check(self.L.rt_get_neighbours(self.ctx, _ptr(ptr), _ptr(idx)))
        return ptr, idx[:st["n_entries"]]

    def rt_get_sources(self):
        st = self.rt_get_stats()
        m = max(st["n_inject"], 1)
        gas = torch.empty(m, dtype=torch.int32, device=self.device)
        src = torch.empty(m, dtype=torch.int32, device=self.device)
        xi = torch.empty(m, dtype=torch.float64, device=self.device)
        hs = torch.empty(max(self.S, 1), dtype=torch.float64, device=self.device)
        self._check(self.L.rt_get_sources(self.ctx, _ptr(gas), _ptr(src), _ptr(xi), _ptr(hs)))
        k = st["n_inject"]
        return gas[:k], src[:k], xi[:k], hs[:self.S]

    def rt_timing(self, on: bool):
        self._bind_stream()
        self._check(self.L.rt_timing(self.ctx, 1 if on else 0))

    def rt_get_timing(self, kernel: str):
        ms = ctypes.c_double()
        cnt = ctypes.c_int64()
        self._check(self.L.rt_get_timing(self.ctx, kernel.encode(), ctypes.byref(ms),
                                         ctypes.byref(cnt)))
        return ms.value, cnt.value

    # -- composition of the entry points (no arithmetic) ----------------------
    def step(self, U: torch.Tensor, L: Optional[torch.Tensor] = None, UD=None, U_out=None,
             **kw) -> torch.Tensor:
        """One RT step in the operator-splitting order injection -> gradient ->
        transport (Part III "One RT time step").  U is injected in place."""
        if self.S:
            self.rt_inject(U, L)
        UD = self.rt_gradient(U, UD)
        return self.rt_transport(UD, U_out=U_out, **kw)
