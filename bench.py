"""Benchmark of the photon transport step on one MI355X.

Workload (default): 2^20 particles on a 128^3 lattice with +-0.1 spacing
jitter in the periodic unit box, 3 photon groups, 16 point sources at random
particles with log-uniform luminosities in [1e-2, 1], reduced speed of light
c = 1, CFL 0.9, FP64.  One step = injection -> gradient -> transport (with the
fused update, guards and photon budget), i.e. one pass of the whole per-step
hot path; the static geometry (Morton sort, smoothing lengths, neighbour
table, volumes, matrices) is built once beforehand and reported separately.

Metric: RT pair interactions per second = (unordered interacting pairs,
r < max(H_k, H_l)) x steps / wall time of the timed steps.

Prints one JSON line (rank 0).  Extra keys: roofline of the transport kernel,
cpu_baseline (the FP64 oracle on a bounded sample of the same recipe), and
per-kernel times.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64_VALU = 78.6e12      # MI355X FP64 vector, FLOP/s
PEAK_FP32_VALU = 157.3e12     # MI355X FP32 vector, FLOP/s
PEAK_HBM = 8.0e12             # bytes/s


def transport_flops_per_pair(G: int) -> int:
    """Algorithmic FP operations of one unordered pair in the transport kernel
    (each pair counted once; fma = 2, sqrt/div = 1): pair geometry 74, per
    group 179 (limited extrapolation of 4 quantities 72, two face guards 16,
    M1 fluxes of both faces 70, GLF and accumulation 21)."""
    return 74 + 179 * G


def transport_bytes_per_particle(G: int, elem: int) -> int:
    """Algorithmic HBM bytes per particle and transport launch: geometry record
    (96 B used of its 128-B line), gradient record read (state 4 G and
    gradients 12 G elements), U_out written (4 G elements)."""
    return 96 + (16 + 4) * G * elem


def src_sha(path: str) -> str:
    return hashlib.sha256(open(path, "rb").read()).hexdigest()[:16]


def log(msg: str):
    print(msg, file=sys.stderr, flush=True)


def cpu_baseline(cfg_index: int, min_seconds: float):
    """The FP64 oracle as it stands, on a bounded sample of the same recipe:
    the 64^3 lattice (same jitter, groups and sources; same neighbour count per
    particle, 1/8 of the particles), timed over whole steps."""
    import oracle
    import workloads
    w = workloads.config(cfg_index, scale=(64 ** 3) / (128 ** 3))
    t0 = time.time()
    geo = oracle.build_geometry(w.x)
    srcs = oracle.build_sources(geo, w.xs)
    log(f"cpu baseline: oracle geometry of {w.n} particles in {time.time() - t0:.1f} s")
    U = w.U0.copy()
    steps, t = 0, 0.0
    while t < min_seconds or steps < 2:
        t1 = time.perf_counter()
        U, _ = oracle.step(geo, srcs, U, w.L)
        t += time.perf_counter() - t1
        steps += 1
    return {
        "value": geo.n_pairs * steps / t,
        "unit": "pair-interactions/s",
        "cores": oracle.num_threads(),
        "kind": "oracle",
        "sample": f"{w.n} particles (64^3 jittered lattice, 3 groups, 16 sources, same recipe), "
                  f"{steps} full steps (inject+gradient+transport) in {t:.1f} s",
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32c"])
    ap.add_argument("--config", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also launch a plain device copy of 1 GiB (HBM counter calibration)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: this build runs on one GPU only; --gpus above 1 is not supported "
              "(multi-GPU sharding is a design note, not an implementation)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import workloads
    from paper_2302_12727_amd import RT

    dev = torch.device("cuda:0")
    w = workloads.config(args.config)
    G = w.groups
    log(f"workload {w.name}: n={w.n} G={G} S={w.xs.shape[0]} precision={args.precision}")

    rt = RT(w.n, G, precision=args.precision, cfl=w.cfl, c_red=w.c_red, device=dev)
    x = torch.from_numpy(w.x).to(dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    perm, h, V, dt = rt.rt_build_cells(x)
    if w.xs.shape[0]:
        rt.rt_set_sources(torch.from_numpy(w.xs).to(dev))
    rt.rt_sync()
    build_ms = (time.perf_counter() - t0) * 1e3
    st = rt.rt_get_stats()
    pairs = st["n_pairs"]
    log(f"build {build_ms:.1f} ms; pairs {pairs}; mean neighbours {st['n_entries'] / w.n:.2f}; "
        f"max {st['max_neighbours']}; device MiB {st['device_bytes'] / 2**20:.0f}")

    p = perm.cpu().numpy()
    sd = torch.float64 if args.precision == "fp64" else torch.float32
    U = torch.from_numpy(np.ascontiguousarray(w.U0[p])).to(dev).to(sd)
    Ub = torch.empty_like(U)
    UD = rt.grad_buffer()
    L = torch.from_numpy(w.L).to(dev)
    Q = torch.zeros(G, dtype=torch.float64, device=dev)
    counts = torch.zeros(4, dtype=torch.int64, device=dev)
    ledger = torch.zeros(G, dtype=torch.float64, device=dev)

    def step(U, Ub):
        if rt.S:
            rt.rt_inject(U, L)
        rt.rt_gradient(U, UD)
        rt.rt_transport(UD, U_out=Ub, photon_total=Q, counts=counts, ledger=ledger)
        return Ub, U

    for _ in range(args.warmup):
        U, Ub = step(U, Ub)
    Q0 = rt.rt_photon_total(U).cpu().numpy()
    ledger.zero_()
    torch.cuda.synchronize()

    rt.rt_timing(True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(args.steps):
        U, Ub = step(U, Ub)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t1
    rt.rt_timing(False)
    rt.rt_sync()
    tr_ms, tr_n = rt.rt_get_timing("transport")
    gr_ms, gr_n = rt.rt_get_timing("gradient")
    in_ms, in_n = rt.rt_get_timing("inject")

    if args.copy_calibration:
        a = torch.empty(1 << 27, dtype=torch.float64, device=dev)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()

    elem = 8 if args.precision == "fp64" else 4
    tr_avg = tr_ms / max(tr_n, 1) * 1e-3
    flops = transport_flops_per_pair(G) * pairs
    peak = PEAK_FP64_VALU if args.precision == "fp64" else PEAK_FP32_VALU
    achieved = flops / tr_avg
    traffic = None
    tf = os.path.join(ROOT, "profiles", f"transport_traffic_{w.name}_{args.precision}.json")
    if os.path.exists(tf):
        rec = json.load(open(tf))
        if rec.get("source_sha") == src_sha(os.path.join(ROOT, "paper_2302_12727_amd", "csrc",
                                                         "rt_step.hip")):
            traffic = rec.get("hbm_bytes_per_launch")

    out = {
        "metric": "RT pair interactions/s (FP64)" if args.precision == "fp64"
                  else "RT pair interactions/s (FP32-compensated)",
        "value": pairs * args.steps / elapsed,
        "unit": "pair-interactions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32",
        "data": "synthetic",
        "config": {"workload": f"{w.name}: 2^20-particle 128^3 jittered lattice, 3 groups, "
                               f"16 sources, c=1, CFL 0.9" if args.config == 1 else w.name,
                   "n": w.n, "groups": G, "sources": int(w.xs.shape[0]),
                   "pairs": pairs, "precision": args.precision},
        "roofline": {"bound": "alu", "kernel": "transport", "achieved": achieved / 1e12,
                     "peak": peak / 1e12, "unit": "TFLOP/s", "frac": achieved / peak,
                     "traffic": traffic,
                     "flops_per_pair": transport_flops_per_pair(G),
                     "algorithmic_bytes_per_launch": transport_bytes_per_particle(G, elem) * w.n,
                     "hbm_frac_at_algorithmic_bytes":
                         transport_bytes_per_particle(G, elem) * w.n / tr_avg / PEAK_HBM},
        "kernel_ms": {"transport": tr_ms / max(tr_n, 1), "gradient": gr_ms / max(gr_n, 1),
                      "inject": in_ms / max(in_n, 1) if in_n else 0.0},
        "build_ms": build_ms,
        # photon budget over the timed steps: Q_end = Q_0 + steps dt sum L + ledger
        "photon_budget_residual": float(np.max(np.abs(
            Q.cpu().numpy() - (Q0 + args.steps * float(dt.item()) * w.L.sum(axis=0)
                               + ledger.cpu().numpy())) / Q.cpu().numpy())),
        "guard_counts": counts.cpu().tolist(),
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args.config, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
