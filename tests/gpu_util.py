"""Helpers shared by the GPU parity tests (no method arithmetic here)."""
import numpy as np
import torch


def dev(a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.to("cuda")


def unsort(a_sorted: np.ndarray, perm: np.ndarray) -> np.ndarray:
    """Morton-ordered rows -> input order."""
    out = np.empty_like(a_sorted)
    out[perm] = a_sorted
    return out


def state_err(got: np.ndarray, ref: np.ndarray, floor_frac: float = 1e-6) -> float:
    """Largest per-particle, per-group error of (E, F) relative to that state's
    magnitude max(E, |F|/c) (floored at floor_frac times the mean energy)."""
    scale = np.maximum(np.abs(ref).max(axis=-1), floor_frac * np.abs(ref[..., 0]).mean())
    return float((np.abs(got - ref).max(axis=-1) / scale).max())


def log(msg):
    print(msg, flush=True)


def local_scale(ref: np.ndarray, sptr: np.ndarray, sidx: np.ndarray) -> np.ndarray:
    """Per particle and group: the largest state magnitude max(E, |F|/c) over the
    particle and its neighbours (oracle CSR lists), c = 1."""
    mag = np.abs(ref).max(axis=-1)                       # [n, G]
    gathered = mag[sidx]                                 # [entries, G]
    n = ref.shape[0]
    out = mag.copy()
    nz = np.diff(sptr) > 0
    red = np.maximum.reduceat(gathered, sptr[:-1][nz], axis=0)
    out[nz] = np.maximum(out[nz], red)
    return out


def local_err(got: np.ndarray, ref: np.ndarray, sptr, sidx) -> float:
    """Largest error of (E, F) relative to the local scale of the neighbourhood."""
    return float((np.abs(got - ref).max(axis=-1) / local_scale(ref, sptr, sidx)).max())


def err_summary(got, ref, sptr, sidx) -> str:
    per = np.abs(got - ref).max(axis=-1) / np.maximum(np.abs(ref).max(axis=-1), 1e-300)
    q = np.quantile(per, [0.5, 0.99, 0.999, 1.0])
    return (f"per-state rel err median {q[0]:.2e} p99 {q[1]:.2e} p99.9 {q[2]:.2e} "
            f"max {q[3]:.2e}; local-scale rel err max {local_err(got, ref, sptr, sidx):.2e}")
