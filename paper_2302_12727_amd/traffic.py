"""HBM traffic of the transport kernel from rocprofv3 counter runs.

Two `rocprofv3 --pmc` runs of `bench.py --copy-calibration` (one with
FETCH_SIZE, one with WRITE_SIZE) give the kernel's counters per dispatch in
KiB.  The same runs launch a plain device copy of 1 GiB; what the counters read
for it calibrates them (on gfx950 the copy reads as 0.5 GiB fetched and
1 GiB written, so fetches are scaled by 2).  The record written here is what
bench.py reports as roofline.traffic, and only while the kernel sources still
hash to the recorded source_sha.

    python -m paper_2302_12727_amd.traffic --fetch DIR --write DIR \\
        --workload NAME --precision fp64 --out FILE.json --command "..."
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os

HERE = os.path.dirname(os.path.abspath(__file__))
COPY_BYTES = 1 << 30


def transport_sources(precision: str):
    """Source files that define the transport kernel of one precision and what
    it reads (the neighbour table and the tile task lists of rt_build.hip)."""
    d = os.path.join(HERE, "csrc")
    names = ["rt_step.hip", "rt_pair.h"] if precision == "fp64" else ["rt_step32.hip", "rt_pair32.h"]
    return [os.path.join(d, f) for f in names + ["rt_internal.h", "rt_build.hip"]]


def source_sha(*paths: str) -> str:
    h = hashlib.sha256()
    for p in paths:
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def _rows(run_dir: str, counter: str):
    files = glob.glob(os.path.join(run_dir, "**", "*counter_collection.csv"), recursive=True)
    if not files:
        raise FileNotFoundError(f"no counter_collection.csv under {run_dir}")
    for f in files:
        with open(f) as fh:
            for r in csv.DictReader(fh):
                if r["Counter_Name"] == counter:
                    yield r["Kernel_Name"], float(r["Counter_Value"])


def kernel_and_copy(run_dir: str, counter: str, kernel: str):
    """Mean counter value per dispatch of `kernel`, and the value of the largest
    copy dispatch (the 1 GiB calibration copy)."""
    vals, copy = [], 0.0
    for name, v in _rows(run_dir, counter):
        if kernel in name:
            vals.append(v)
        elif "copyBuffer" in name:
            copy = max(copy, v)
    if not vals or copy <= 0:
        raise ValueError(f"{counter}: kernel {kernel!r} or the calibration copy missing in {run_dir}")
    return sum(vals) / len(vals), len(vals), copy


def record(fetch_dir: str, write_dir: str, workload: str, precision: str, command: str) -> dict:
    kernel = "k_transport64" if precision == "fp64" else "k_transport32"
    f, nf, cf = kernel_and_copy(fetch_dir, "FETCH_SIZE", kernel)
    w, nw, cw = kernel_and_copy(write_dir, "WRITE_SIZE", kernel)
    ff, fw = COPY_BYTES / (cf * 1024), COPY_BYTES / (cw * 1024)
    return {
        "workload": workload, "precision": precision, "kernel": kernel,
        "fetch_kib_per_launch": f, "write_kib_per_launch": w, "dispatches": [nf, nw],
        "copy_fetch_kib": cf, "copy_write_kib": cw, "fetch_factor": ff, "write_factor": fw,
        "hbm_bytes_per_launch": f * 1024 * ff + w * 1024 * fw,
        "source_sha": source_sha(*transport_sources(precision)),
        "command": command,
    }


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--fetch", required=True, help="rocprofv3 output folder of the FETCH_SIZE run")
    ap.add_argument("--write", required=True, help="rocprofv3 output folder of the WRITE_SIZE run")
    ap.add_argument("--workload", required=True)
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32c"])
    ap.add_argument("--out", required=True)
    ap.add_argument("--command", default="", help="the profiled command, for the record")
    a = ap.parse_args()
    rec = record(a.fetch, a.write, a.workload, a.precision, a.command)
    with open(a.out, "w") as fh:
        json.dump(rec, fh, indent=1)
    print(json.dumps(rec))


if __name__ == "__main__":
    main()
