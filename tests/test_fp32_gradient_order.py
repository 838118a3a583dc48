"""Why the compensated-FP32 adjoint moves with the FP32 gradient's lane
order: a NumPy float32 emulation of the FP32 gradient's sums (eq:gradient) in
the two orders the kernel can take (one lane per particle summing its
neighbours in list order; four lanes each summing every fourth neighbour,
joined by a fixed butterfly), on the 1000-particle lattice of the GPU adjoint
tests (2 groups).

Both orders are equally accurate against the FP64 oracle.  But the limiter
of the next transport (minmod of the two sides' projected gradients) meets
one pair whose two slopes agree to 2.5e-7 in FP64, closer than FP32 rounding
of the gradients, and the four-lane order decides it the other way.  An
adjoint differentiates through the branch its forward took, so that single
pair moves the FP32 adjoint's luminosity gradient away from the FP64 one
(1.4e-5 with four lanes against 3e-8 with one, on the GPU): a limiter tie,
not an error of either kernel.  The emulation takes the oracle's neighbour
order and contracts every multiply-add into one rounding, as the GPU does.
"""
import numpy as np

import oracle
import workloads

f32 = np.float32
SIGMA3 = 16.0 / np.pi


def fma32(a, b, c):
    """float32 a * b + c with one rounding (the product is exact in float64)."""
    return (a.astype(np.float64) * b.astype(np.float64) + c.astype(np.float64)).astype(f32)


def grad32(geo, U, lanes):
    """The FP32 gradient record's gradients, [n][G][4][3], summed in the
    order of `lanes` lanes per particle."""
    n, G = U.shape[0], U.shape[1]
    box = float(geo.box[0])
    cnt = np.diff(geo.gptr)
    kmax = int(cnt.max())
    U32 = U.astype(f32).reshape(n, 4 * G)
    iH = (1.0 / geo.H).astype(f32)
    acc = np.zeros((lanes, n, 4 * G, 3), dtype=f32)
    rows = np.arange(n)
    for k in range(kmax):
        live = cnt > k
        i = rows[live]
        j = geo.gidx[geo.gptr[i] + k]
        s = geo.x[j] - geo.x[i]
        s = (s - box * np.rint(s / box)).astype(f32)
        r2 = (s[:, 0] * s[:, 0] + s[:, 1] * s[:, 1]) + s[:, 2] * s[:, 2]
        q = np.sqrt(r2) * iH[i]
        a = np.maximum(f32(1) - q, f32(0))
        b = np.maximum(f32(0.5) - q, f32(0))
        w = a * a * a - f32(4) * (b * b * b)
        ws = w[:, None] * s
        d = U32[j] - U32[i]
        sub = k % lanes
        acc[sub, i] = fma32(d[:, :, None], ws[:, None, :], acc[sub, i])
    t = acc[0] if lanes == 1 else (acc[0] + acc[1]) + (acc[2] + acc[3])
    Sinv = (geo.B * (SIGMA3 / geo.H ** 3 * geo.V)[:, None, None]).astype(f32)
    D = (Sinv[:, None, :, 0] * t[:, :, 0:1] + Sinv[:, None, :, 1] * t[:, :, 1:2]) \
        + Sinv[:, None, :, 2] * t[:, :, 2:3]
    return D.reshape(n, G, 4, 3)


def slopes(geo, D):
    """Both sides' projected gradients of every pair entry, group and component."""
    box = float(geo.box[0])
    sk = np.repeat(np.arange(geo.n), np.diff(geo.sptr))
    sl = geo.sidx
    s = geo.x[sl] - geo.x[sk]
    s = s - box * np.rint(s / box)
    dk = np.einsum("egma,ea->egm", D[sk].astype(np.float64), s)
    dl = np.einsum("egma,ea->egm", D[sl].astype(np.float64), s)
    return dk, dl


def test_lane_order_flips_one_limiter_tie():
    w = workloads.lattice_workload(10, 2, 3, 6, seed=555, name="adj")
    geo = oracle.build_geometry(w.x)
    D64 = oracle.gradient(geo, w.U0)
    scale = np.abs(D64).max(axis=(-1, -2), keepdims=True)
    dk, dl = slopes(geo, D64)
    same = dk * dl > 0
    pick = np.abs(dk) <= np.abs(dl)
    gap = np.abs(np.abs(dk) - np.abs(dl)) / np.maximum(np.abs(dk), np.abs(dl))
    ties = np.argwhere(same & (gap < 1e-6))
    # one pair, seen from both sides, is a limiter tie within FP32 rounding
    assert len(ties) == 2 and 1e-7 < gap[tuple(ties[0])] < 5e-7
    flips = {}
    for lanes in (1, 4):
        D = grad32(geo, w.U0, lanes)
        err = np.abs(D - D64) / scale
        assert err.max() < 1e-5 and np.median(err) < 2e-7
        d32k, d32l = slopes(geo, D)
        assert np.array_equal(d32k * d32l > 0, same)         # no sign decision moves
        moved = np.argwhere(same & ((np.abs(d32k) <= np.abs(d32l)) != pick))
        flips[lanes] = {tuple(e) for e in moved}
    tie_set = {tuple(e) for e in ties}
    assert flips[1] == set()
    assert flips[4] == tie_set
