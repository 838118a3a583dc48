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
