"""Summarise rocprofv3 PMC runs of the benchmark into HBM bytes per launch
and VALU figures per sweep kernel.

FETCH_SIZE and WRITE_SIZE are scaled by what the same counters read for the
calibration copy kernel, which moves a known 4 GiB in and 4 GiB out per
dispatch.  VALU utilisation is the kernel's VALU lane-instructions
(SQ_INSTS_VALU x 64) over its average launch duration from a kernel trace
of the same command, against the issue peak of the chip (256 CUs x 4 SIMDs
x 16 lanes x 2.4 GHz = 39.3e12 lane-instructions/s); it cannot exceed 1.
Usage (from the repository root, after the runs):

    python -m paper_2502_18624_amd.pmc_summary <dir with fetch/ write/ cfetch/ cwrite/> [<dir with valu/> [<kernel_stats.csv>]]

The second directory holds a run with the VALU and LDS counters
(SQ_INSTS_VALU SQ_ACTIVE_INST_VALU SQ_INSTS_LDS SQ_LDS_BANK_CONFLICT SQ_WAVES
SQ_BUSY_CYCLES GRBM_GUI_ACTIVE); the kernel-stats file is the
rocprofv3 --kernel-trace --stats summary of the same command.
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


# The three sweep kernels of the benchmark: name prefix, lattice side, and
# algorithmic bytes per launch (read the own plane, read the other plane,
# write the own plane: 3 L^2 / 2 cells x bits / 8).
SWEEP_KERNELS = {
    "ising_4bit": ("half_sweep_kernel<0, ", 2 ** 17, 4),
    "blume_capel_4bit": ("half_sweep_kernel<1, ", 2 ** 16, 4),
    "ising_1bit": ("lut_half_kernel<", 2 ** 17, 1),
}


# MI355X: 8 XCDs of 32 CUs, 4 SIMDs of 16 lanes per CU; a wave64 VALU
# instruction occupies its SIMD for 4 cycles.  GRBM_GUI_ACTIVE is summed
# over the XCDs.
N_XCD, N_CU, N_SIMD = 8, 256, 1024


def per_kernel_counters(path):
    d = collections.defaultdict(lambda: collections.defaultdict(list))
    for r in csv.DictReader(open(path)):
        d[short(r["Kernel_Name"])][r["Counter_Name"]].append(float(r["Counter_Value"]))
    return {k: {c: sum(v) / len(v) for c, v in cs.items()} for k, cs in d.items()}


VALU_PEAK_LANE_INSTS = N_SIMD * 16 * 2.4e9


def kernel_durations(stats_csv):
    """Average launch duration (seconds) per shortened kernel name from a
    rocprofv3 --stats kernel_stats.csv."""
    out = {}
    for r in csv.DictReader(open(stats_csv)):
        out[short(r["Name"])] = float(r["AverageNs"]) * 1e-9
    return out


def valu_summary(path, durations=None):
    """VALU issue and LDS figures per sweep kernel from a run with SQ_INSTS_VALU,
    SQ_INSTS_LDS, SQ_LDS_BANK_CONFLICT, SQ_WAVES and GRBM_GUI_ACTIVE; with the
    launch durations of a kernel trace, also the VALU utilisation."""
    c = per_kernel_counters(path)
    out = {}
    for name, (prefix, L, bits) in SWEEP_KERNELS.items():
        ks = [k for k in c if k.startswith(prefix)]
        if not ks:
            continue
        m = {n: sum(c[k][n] for k in ks) / len(ks) for n in c[ks[0]]}
        cycles = m["GRBM_GUI_ACTIVE"] / N_XCD
        updates = L * L / 2
        out[name] = {"valu_wave_insts_per_launch": m["SQ_INSTS_VALU"],
                     "valu_lane_ops_per_update": m["SQ_INSTS_VALU"] * 64 / updates,
                     "gpu_cycles_per_launch": cycles,
                     "lds_insts_per_launch": m["SQ_INSTS_LDS"],
                     "lds_bank_conflict_share": m["SQ_LDS_BANK_CONFLICT"] / N_CU / cycles,
                     "waves": m["SQ_WAVES"]}
        if durations:
            ds = [durations[k] for k in ks if k in durations]
            if ds:
                dur = sum(ds) / len(ds)
                out[name]["avg_launch_s"] = dur
                out[name]["valu_util"] = m["SQ_INSTS_VALU"] * 64 / (dur * VALU_PEAK_LANE_INSTS)
    return out


def main(d, valu_dir=None, stats_csv=None):
    f = per_kernel(os.path.join(d, "fetch", "bench_counter_collection.csv"))
    w = per_kernel(os.path.join(d, "write", "bench_counter_collection.csv"))
    cf = per_kernel(os.path.join(d, "cfetch", "copy_counter_collection.csv"))
    cw = per_kernel(os.path.join(d, "cwrite", "copy_counter_collection.csv"))
    copy_kib = 4 * 1024 * 1024
    fs, ws = copy_kib / cf["copy_kernel"], copy_kib / cw["copy_kernel"]
    kernels = {}
    for name, (prefix, L, bits) in SWEEP_KERNELS.items():
        hs = [k for k in f if k.startswith(prefix)]
        if not hs:
            continue
        fetch = sum(f[k] for k in hs) / len(hs) * fs * 1024
        write = sum(w.get(k, 0.0) for k in hs) / len(hs) * ws * 1024
        alg = 3 * L * L * bits / 8 / 2
        kernels[name] = {"kernels": hs, "L": L, "bits_per_cell": bits, "hbm_read_bytes_per_launch": fetch,
                         "hbm_write_bytes_per_launch": write, "hbm_bytes_per_launch": fetch + write,
                         "algorithmic_bytes_per_launch": alg, "traffic_over_algorithmic": (fetch + write) / alg}
    if valu_dir:
        durations = kernel_durations(stats_csv) if stats_csv else None
        for name, v in valu_summary(os.path.join(valu_dir, "valu", "bench_counter_collection.csv"),
                                    durations).items():
            kernels.setdefault(name, {}).update(v)
    return {"kernel_source_sha": source_sha(), "fetch_scale": fs, "write_scale": ws, "sweep_kernels": kernels,
            "per_kernel_bytes": {k: [f[k] * fs * 1024, w.get(k, 0.0) * ws * 1024] for k in f}}


if __name__ == "__main__":
    print(json.dumps(main(sys.argv[1], sys.argv[2] if len(sys.argv) > 2 else None,
                          sys.argv[3] if len(sys.argv) > 3 else None), indent=1))
