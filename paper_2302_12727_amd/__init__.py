"""MI355X (gfx950) implementation of the Gear-RT photon transport step.

The transport step of the particle-based M1 radiative transfer of
arXiv:2302.12727 (Part III) on the Hopkins finite volume particle method
(Part II), as a C-ABI HIP library (include/rt.h, libgearrt.so) with a thin
torch binding (`rt.RT`) and a differentiable rollout (`rollout.RTRollout`).
"""
from .rt import RT, RTError, load_library, hll_speed_table, photon_groups, KAPPA, ETA  # noqa: F401

__all__ = ["RT", "RTError", "load_library", "hll_speed_table", "photon_groups", "KAPPA",
           "ETA"]
