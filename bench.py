"""Benchmark: checkerboard Metropolis quench of the 2D Ising model on one
MI355X, L = 2^17 (1.7e10 spins, 4-bit cells, 8 GiB), random +-1 start,
quench to T = T_c, C(r, t) (protocol mode, both axes) plus B, M, Q at every
t = 2^k, one lattice per launch.  A step is one sweep (and the measurement
when t reaches a power of two).  Prints one JSON line.

    python bench.py [--gpus 1] [--steps 2000] [--warmup 10]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

BETA_C = math.log(1.0 + math.sqrt(2.0)) / 2.0
HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, published
METRIC = "lattice updates/ns on 1 MI355X (Ising L=2^17); % HBM peak; batched vs plain"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_baseline(budget_s=12.0):
    """The oracle on the host cores: Ising at T_c from a random start on an
    L = 2^13 sample of the workload, whole sweeps until ~budget_s elapse."""
    import oracle
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        cores = os.cpu_count() or 1
    L = 2 ** 13
    s = oracle.init(oracle.ISING, L, 1002)
    done, t0 = 0, time.perf_counter()
    while True:
        oracle.sweep(s, oracle.ISING, 1002, done, 1, BETA_C, 0.0, nthreads=cores)
        done += 1
        el = time.perf_counter() - t0
        if el > budget_s or done >= 16:
            break
    return {"value": round(L * L * done / (el * 1e9), 5), "unit": "updates/ns", "cores": cores, "kind": "oracle",
            "sample": "Ising L=2^13 at T_c from a random start, %d sweeps (%.1f s), rows of one colour split over "
                      "%d OpenMP threads" % (done, el, cores)}


def run(args):
    import torch

    import paper_2502_18624_amd as mcl

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream(dev)
    L, seed, beta = args.L, 1002, BETA_C
    log("bench: Ising L=%d, %d warmup + %d timed sweeps" % (L, args.warmup, args.steps))
    lat = mcl.Lattice(mcl.ISING, L, seed, stream=stream)
    if args.warmup:
        lat.sweep(args.warmup, beta)
        lat.measure(mcl.CORR_PROTOCOL)
        torch.cuda.synchronize()
    mem = lat.mem
    lat.free()
    lat = mcl.Lattice(mcl.ISING, L, seed, stream=stream, mem=mem)   # quench restarts at t = 0
    torch.cuda.synchronize()

    marks = []
    t = 1
    while t <= args.steps:
        marks.append(t)
        t *= 2
    ev = []
    measures = []
    t_meas = 0.0
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    done = 0
    for m in marks + [args.steps]:
        if m > done:
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record(stream)
            lat.sweep(m - done, beta)
            b.record(stream)
            ev.append((a, b, m - done))
            done = m
        if m in marks and (not measures or measures[-1]["t"] != m):
            tm = time.perf_counter()
            out = lat.measure(mcl.CORR_PROTOCOL)
            t_meas += time.perf_counter() - tm
            measures.append({"t": out["t"], "B": out["B"], "M": out["M"], "n_r": int(len(out["r"])),
                             "Cx1": int(out["Cx"][1]), "Cy1": int(out["Cy"][1])})
            log("  t=%d B=%d M=%d" % (out["t"], out["B"], out["M"]))
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    sweep_ms = sum(a.elapsed_time(b) for a, b, _ in ev)
    n_sweeps = sum(k for _, _, k in ev)
    assert n_sweeps == args.steps and lat.t == args.steps
    updates = float(L) * L * args.steps
    half_ms = sweep_ms / (2 * n_sweeps)
    half_bytes = 3.0 * L * L / 4.0                 # read P_c, read P_{1-c}, write P_c (4-bit cells)
    achieved = half_bytes / (half_ms * 1e-3) / 1e9
    res = {
        "metric": METRIC,
        "value": round(updates / (wall * 1e9), 2),
        "unit": "updates/ns",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall * 1e3 / args.steps, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u4 (4-bit spin cells, u32 Philox draws)",
        "data": "synthetic (seeded Philox4x32-10 random start)",
        "config": {"workload": "Ising quench, L=2^17, T=T_c, random +-1 start, %d sweeps, protocol C(r,t) and "
                               "B/M at t=2^k, one lattice per launch" % args.steps,
                   "L": L, "seed": seed, "beta": beta, "measure_times": marks},
        "sweep_only_updates_per_ns": round(updates / (sweep_ms * 1e6), 2),
        "measure_share": round(t_meas / wall, 4),
        "hbm_frac": round(achieved / HBM_PEAK_GBS, 4),
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                     "kernel": "half_sweep_kernel<Ising>", "avg_launch_ms": round(half_ms, 4),
                     "bytes_per_launch": half_bytes},
        "paper_context": {"updates_per_ns": 1797, "hardware": "1x GB200, 1-bit cells with LUT random bits",
                          "note": "context only"},
        "measures": measures,
    }
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--L", type=int, default=2 ** 17)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path (got --gpus %d)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)
    res = run(args)
    if not args.no_cpu_baseline:
        log("bench: timing the CPU oracle sample")
        res["cpu_baseline"] = cpu_baseline()
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
