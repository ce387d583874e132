"""Summarise rocprofv3 PMC runs of the benchmark into HBM bytes per launch.

FETCH_SIZE and WRITE_SIZE are scaled by what the same counters read for the
calibration copy kernel, which moves a known 4 GiB in and 4 GiB out per
dispatch.  Usage (from the repository root, after the four PMC runs):

    python -m paper_2502_18624_amd.pmc_summary <dir with fetch/ write/ cfetch/ cwrite/> <L>
"""
from __future__ import annotations

import collections
import csv
import hashlib
import json
import os
import re
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
KERNEL_SOURCES = ["paper_2502_18624_amd/csrc/sweep.hip", "paper_2502_18624_amd/csrc/sweep_device.h",
                  "paper_2502_18624_amd/csrc/common.h"]


def short(name):
    m = re.search(r"(\w+_kernel(<[^>]*>)?|__amd_\w+)", name)
    return m.group(1) if m else name[:40]


def per_kernel(path):
    d = collections.defaultdict(list)
    for r in csv.DictReader(open(path)):
        d[short(r["Kernel_Name"])].append(float(r["Counter_Value"]))
    return {k: sum(v) / len(v) for k, v in d.items()}


def source_sha():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def main(d, L):
    f = per_kernel(os.path.join(d, "fetch", "bench_counter_collection.csv"))
    w = per_kernel(os.path.join(d, "write", "bench_counter_collection.csv"))
    cf = per_kernel(os.path.join(d, "cfetch", "copy_counter_collection.csv"))
    cw = per_kernel(os.path.join(d, "cwrite", "copy_counter_collection.csv"))
    copy_kib = 4 * 1024 * 1024
    fs, ws = copy_kib / cf["copy_kernel"], copy_kib / cw["copy_kernel"]
    hs = [k for k in f if k.startswith("half_sweep_kernel<0, true")]
    fetch = sum(f[k] for k in hs) / len(hs) * fs * 1024
    write = sum(w[k] for k in hs) / len(hs) * ws * 1024
    alg = 3 * L * L / 4
    rec = {"kernel": "half_sweep_kernel<Ising> (mean of both colours)", "L": L, "kernel_source_sha": source_sha(),
           "fetch_scale": fs, "write_scale": ws, "hbm_read_bytes_per_launch": fetch,
           "hbm_write_bytes_per_launch": write, "hbm_bytes_per_launch": fetch + write,
           "algorithmic_bytes_per_launch": alg, "traffic_over_algorithmic": (fetch + write) / alg,
           "per_kernel_bytes": {k: [f[k] * fs * 1024, w.get(k, 0.0) * ws * 1024] for k in f}}
    return rec


if __name__ == "__main__":
    print(json.dumps(main(sys.argv[1], int(sys.argv[2])), indent=1))
