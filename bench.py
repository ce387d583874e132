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
# VALU peak: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz = 39.3e12 32-bit lane
# instructions/s.  One Philox4x32-10 block needs 10 rounds x (2 wide
# multiplies + 2 three-input xors) = 40 of them at the least on gfx950.
VALU_LANE_OPS = 256 * 64 * 2.4e9
PHILOX_OPS_PER_BLOCK = 40
PHILOX_PEAK_GBLOCKS = VALU_LANE_OPS / PHILOX_OPS_PER_BLOCK / 1e9
METRIC = "lattice updates/ns on 1 MI355X (Ising L=2^17); % HBM peak; batched vs plain"
SWEEP_SOURCES = ["paper_2502_18624_amd/csrc/sweep.hip", "paper_2502_18624_amd/csrc/sweep_device.h",
                 "paper_2502_18624_amd/csrc/common.h"]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def host_cpu():
    """CPU model (lscpu's "Model name", read from /proc/cpuinfo), nproc and
    the cores this process may run on."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.lower().startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        cores = os.cpu_count() or 1
    return {"model": model, "nproc": os.cpu_count(), "cores": cores}


def _time_oracle_sweeps(model, L, seed, n, beta, D, threads):
    """Seconds of n oracle sweeps of a T = infinity start (i.i.d. +-1, or
    uniform over -1/0/+1 for Blume-Capel), drawn here with numpy: the sweep's
    cost does not depend on which sample it gets, and the oracle's own
    initialisation (one Philox block per site, one thread) would take longer
    than the sweeps."""
    import numpy as np

    import oracle
    rng = np.random.default_rng(seed)
    vals = np.array([-1, 0, 1] if model == oracle.BC else [-1, 1], dtype=np.int8)
    s = vals[rng.integers(0, len(vals), size=(L, L))]
    t0 = time.perf_counter()
    oracle.sweep(s, model, seed, 0, n, beta, D, nthreads=threads)
    return time.perf_counter() - t0


def _time_oracle_quench(threads):
    """The parity-size workload in full: Ising L = 256, seed 1001, 0.9 T_c,
    random start, 1000 sweeps, B/M and full C(r) along both axes at t = 2^k."""
    import oracle
    L, seed, beta, total = 256, 1001, BETA_C / 0.9, 1000
    s = oracle.init(oracle.ISING, L, seed)
    t0 = time.perf_counter()
    done = 0
    for t in oracle.schedule_pow2(total) + [total]:
        oracle.sweep(s, oracle.ISING, seed, done, t - done, beta, nthreads=threads)
        done = t
        if t < total:
            oracle.measure(s, threads)
            oracle.corr(s, oracle.CORR_FULL, oracle.rset(oracle.CORR_FULL, L, t), threads)
    return time.perf_counter() - t0


def cpu_baseline(full=False):
    """The oracle timed on the host cores, single-threaded and with the rows
    of one colour split over every core (same results either way):
    - the parity-size workload in full (Ising L = 256, 1000 sweeps, full C(r)
      at t = 2^k), both ways;
    - Ising at T_c, one sweep: L = 2^15 on all cores (value = this rate, the
      headline workload's update at a size the oracle sweeps in seconds) and
      L = 2^14 on one thread;
    - Blume-Capel at T = 1.4, D = 1, one sweep of L = 2^15 on all cores.
    With full, the whole timing plan instead: Ising L = 2^15 and 2^17 (one
    sweep) and Blume-Capel L = 2^16 (two sweeps), each both ways (about ten
    minutes of single-threaded sweeps)."""
    import oracle
    cpu = host_cpu()
    n_all = cpu["cores"]
    legs = []

    def leg(name, updates, secs, threads):
        legs.append({"workload": name, "threads": threads, "seconds": round(secs, 3),
                     "updates_per_ns": round(updates / (secs * 1e9), 5)})
        log("  oracle %s, %d thread(s): %.2f s" % (name, threads, secs))

    def ising(L, th):
        leg("Ising L=2^%d at T_c, 1 sweep" % int(math.log2(L)), float(L) * L,
            _time_oracle_sweeps(oracle.ISING, L, 1002, 1, BETA_C, 0.0, th), th)

    def bc(L, n, th):
        leg("Blume-Capel L=2^%d, T=1.4, D=1, %d sweep(s)" % (int(math.log2(L)), n), float(L) * L * n,
            _time_oracle_sweeps(oracle.BC, L, 1003, n, 1 / 1.4, 1.0, th), th)

    for th in (1, n_all):
        leg("Ising L=256, 1000 sweeps, full C(r) at t=2^k", 256.0 * 256 * 1000, _time_oracle_quench(th), th)
    ising(2 ** 15, n_all)
    head = legs[-1]
    if full:
        ising(2 ** 15, 1)
        for th in (n_all, 1):
            ising(2 ** 17, th)
        for th in (n_all, 1):
            bc(2 ** 16, 2, th)
    else:
        ising(2 ** 14, 1)
        bc(2 ** 15, 1, n_all)
    single = next(x for x in legs if x["workload"].startswith("Ising L=2^1") and x["threads"] == 1)
    return {"value": head["updates_per_ns"], "unit": "updates/ns", "cores": n_all, "kind": "oracle",
            "sample": "%s with the rows of one colour split over %d OpenMP threads; legs lists every timing"
                      % (head["workload"], n_all),
            "single_thread_value": single["updates_per_ns"], "single_thread_sample": single["workload"],
            "cpu_model": cpu["model"], "nproc": cpu["nproc"], "legs": legs}


def kernel_source_sha():
    import hashlib
    h = hashlib.sha256()
    for f in SWEEP_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def profile_record(name):
    """PMC figures of a sweep kernel ("ising_4bit", "blume_capel_4bit",
    "ising_1bit") from the committed summary, if they were taken on the
    current kernel source (else None)."""
    path = os.path.join(ROOT, "profiles", "traffic_sweep_kernels.json")
    try:
        with open(path) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    if rec.get("kernel_source_sha") != kernel_source_sha():
        return None
    return rec.get("sweep_kernels", {}).get(name)


def measured_traffic(name):
    """HBM bytes per launch from the committed PMC summary (or None)."""
    k = profile_record(name)
    return None if k is None else round(k["hbm_bytes_per_launch"])


def traffic_source():
    """Where roofline.traffic comes from, and whether it applies to the
    kernel source being timed."""
    path = os.path.join(ROOT, "profiles", "traffic_sweep_kernels.json")
    try:
        with open(path) as f:
            sha = json.load(f).get("kernel_source_sha")
    except (OSError, ValueError):
        return "no PMC summary found (profiles/traffic_sweep_kernels.json)"
    state = "current" if sha == kernel_source_sha() else "stale: kernel source changed since, traffic null"
    return "rocprofv3 --pmc FETCH_SIZE, WRITE_SIZE (profiles/traffic_sweep_kernels.md), kernel source %s: %s" % (
        sha, state)


def measured_valu_util(name):
    """VALU lane-instructions of a launch over its duration, as a fraction of
    the chip's issue peak (PMC and kernel trace), or None."""
    k = profile_record(name)
    return None if k is None or "valu_util" not in k else round(k["valu_util"], 3)


def _calibrate(mode):
    """Output of the calibration program in one mode ("copy" or "philox"), or ""."""
    import subprocess
    exe = os.path.join(ROOT, "paper_2502_18624_amd", "mcl_calibrate")
    if not os.path.exists(exe):
        return ""
    try:
        return subprocess.run([exe, mode], capture_output=True, text=True, timeout=60).stdout
    except (OSError, subprocess.SubprocessError):
        return ""


def attainable_copy():
    """Copy-kernel bandwidth from the calibration program (GB/s), or None."""
    import re
    vals = [float(v) for v in re.findall(r"copy .*?([0-9.]+) GB/s", _calibrate("copy"))]
    return max(vals) if vals else None


def attainable_philox():
    """Philox4x32-10 blocks/s of the library's Philox alone, from the
    calibration program (Gblocks/s), or None."""
    import re
    m = re.search(r"philox attainable: ([0-9.]+) Gblocks/s", _calibrate("philox"))
    return float(m.group(1)) if m else None


def replica_set(n=512, seed=3):
    """Batched workload: n replicas alternating Ising / Blume-Capel, L uniform
    over {512 ... 8192}, T ~ U[0.5, 1.5] T_c, D in {0, 0.5, 1} (Blume-Capel),
    replica i seeded 2000 + i; parameters from numpy default_rng(seed)."""
    import numpy as np
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        model = i % 2
        L = int(rng.choice([512, 1024, 2048, 4096, 8192]))
        T = float(rng.uniform(0.5, 1.5)) / BETA_C
        D = float(rng.choice([0.0, 0.5, 1.0])) if model == 1 else 0.0
        out.append((model, L, 2000 + i, 1.0 / T, D))
    return out


def quench_leg(model, L, seed, beta, D, n, half_bytes, blocks_per_update, label, traffic_key):
    """One lattice quenched from its random start and relaxed for n sweeps,
    with B/M/Q and protocol C(r,t) at t = 2^k; whole-job and sweep-only
    rates, the average half-sweep and its HBM and Philox fractions."""
    import torch

    import paper_2502_18624_amd as mcl
    stream = torch.cuda.current_stream()
    lat = mcl.Lattice(model, L, seed, stream=stream)
    lat.sweep(2, beta, D)                            # warm-up, then restart the quench
    torch.cuda.synchronize()
    mem = lat.mem
    lat.free()
    lat = mcl.Lattice(model, L, seed, stream=stream, mem=mem)
    torch.cuda.synchronize()
    marks = [2 ** k for k in range(20) if 2 ** k <= n]
    ev, done, t_meas = [], 0, 0.0
    wall0 = time.perf_counter()
    last = None
    for m in marks + [n]:
        if m > done:
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            lat.sweep(m - done, beta, D)
            b.record(stream)
            ev.append((a, b, m - done))
            done = m
        if m in marks and (last is None or last != m):
            torch.cuda.synchronize()
            tm = time.perf_counter()
            out = lat.measure(mcl.CORR_PROTOCOL)
            t_meas += time.perf_counter() - tm
            last = m
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    sweep_ms = sum(a.elapsed_time(b) for a, b, _ in ev)
    upd = float(L) * L * n
    half_s = sweep_ms / (2 * n) * 1e-3
    gblocks = L * L / 2.0 * blocks_per_update / half_s / 1e9
    res = {"workload": label,
           "updates_per_ns": round(upd / (wall * 1e9), 2),
           "sweep_only_updates_per_ns": round(upd / (sweep_ms * 1e6), 2),
           "avg_half_sweep_ms": round(sweep_ms / (2 * n), 4),
           "hbm_frac": round(half_bytes / half_s / 1e9 / HBM_PEAK_GBS, 4),
           "philox_frac": round(gblocks / PHILOX_PEAK_GBLOCKS, 4),
           "hbm_traffic_bytes_per_launch": measured_traffic(traffic_key),
           "valu_util_pmc": measured_valu_util(traffic_key),
           "algorithmic_bytes_per_launch": half_bytes,
           "measure_share": round(t_meas / wall, 4),
           "final": {"t": out["t"], "B": out["B"], "M": out["M"], "Q": out["Q"],
                     "schwinger_dyson": round(mcl.schwinger_dyson(out["sd"], beta), 7)}}
    lat.free()
    return res


def run_blume_capel(args):
    """Blume-Capel quench, L = 2^16, T = 1.4, D = 1, random start."""
    import paper_2502_18624_amd as mcl
    L, n = 2 ** 16, args.bc_sweeps
    # a half-sweep reads both 4-bit planes and writes one: 3 L^2 / 4 bytes;
    # one u32 acceptance draw plus one proposal bit per update
    res = quench_leg(mcl.BC, L, 1003, 1 / 1.4, 1.0, n, 3.0 * L * L / 4.0, 0.25 + 1.0 / 128,
                     "Blume-Capel quench, L=2^16, T=1.4, D=1.0, random start, %d sweeps, protocol C(r,t) and "
                     "B/M/Q at t=2^k" % n, "blume_capel_4bit")
    res["paper_context_updates_per_ns"] = 941
    return res


def run_ising_1bit(args):
    """Ising with one bit per spin and table-driven random bits, L = 2^17,
    T = T_c, random start: the paper's own Ising kernel design."""
    import paper_2502_18624_amd as mcl
    L, n = 2 ** 17, args.lut_sweeps
    # 1-bit planes: 3 L^2 / 16 bytes per half-sweep; two u32 draws per group
    # of 4 sites (exp4 and exp8 bits) = 1/8 Philox block per update
    res = quench_leg(mcl.ISING_LUT, L, 1002, BETA_C, 0.0, n, 3.0 * L * L / 16.0, 1.0 / 8,
                     "Ising 1-bit (table-driven random bits), L=2^17, T=T_c, random start, %d sweeps, protocol "
                     "C(r,t) and B/M at t=2^k" % n, "ising_1bit")
    res["paper_context_updates_per_ns"] = 1797
    return res


# Single-GPU throughput against L (the paper's Tables 1 and 2; GB200
# figures, context only).
PAPER_TABLE_ISING_1BIT = {13: 1051, 14: 1530, 15: 1741, 16: 1784, 17: 1797, 18: 1801, 19: 1802, 20: 1802}
PAPER_TABLE_BC = {12: 304, 13: 633, 14: 839, 15: 922, 16: 941, 17: 947, 18: 949, 19: 948}


def run_scan(args):
    """Sweep-only updates/ns against L for the three models: random start,
    T = T_c (Blume-Capel T = 1.4, D = 1), about 2e12 updates per size, HIP
    events around the sweep calls; sizes that do not fit the free device
    memory are skipped."""
    import gc

    import torch

    import paper_2502_18624_amd as mcl
    stream = torch.cuda.current_stream()
    gc.collect()
    torch.cuda.empty_cache()                             # earlier legs' cached blocks
    legs = [(mcl.ISING_LUT, range(13, 21), BETA_C, 0.0, PAPER_TABLE_ISING_1BIT),
            (mcl.BC, range(12, 20), 1 / 1.4, 1.0, PAPER_TABLE_BC),
            (mcl.ISING, range(12, 20), BETA_C, 0.0, {})]
    names = {mcl.ISING_LUT: "ising_1bit", mcl.BC: "blume_capel", mcl.ISING: "ising_4bit"}
    out = {}
    for model, ks, beta, D, paper in legs:
        rows = []
        for k in ks:
            L = 2 ** k
            free, _ = torch.cuda.mem_get_info()
            if mcl.query_bytes(model, L) + (1 << 30) > free:
                rows.append({"log2L": k, "skipped": "does not fit the free device memory"})
                continue
            n = max(2, int(round(args.scan_updates / float(L * L))))
            lat = mcl.Lattice(model, L, 7 + k, stream=stream)
            lat.sweep(2, beta, D)                        # warm-up
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            lat.sweep(n, beta, D)
            b.record(stream)
            b.synchronize()
            ms = a.elapsed_time(b)
            rec = {"log2L": k, "sweeps": n, "updates_per_ns": round(float(L) * L * n / (ms * 1e6), 1)}
            if k in paper:
                rec["paper_gb200"] = paper[k]
            rows.append(rec)
            log("  scan %s L=2^%d: %.1f updates/ns" % (names[model], k, rec["updates_per_ns"]))
            lat.free()
            del lat
            gc.collect()
            torch.cuda.empty_cache()
        out[names[model]] = rows
    out["workload"] = ("one lattice per size, random start, T = T_c (Blume-Capel T = 1.4, D = 1), about %.0e "
                       "updates per size, sweep-only (HIP events)" % args.scan_updates)
    return out


def run_batched(args):
    """Batched vs plain on the same replica set: group_sweep (autotuned) and
    one lattice per launch, sweep by sweep."""
    import torch

    import paper_2502_18624_amd as mcl
    from paper_2502_18624_amd.autotune import autotune_group
    specs = replica_set(args.replicas)
    n = args.batched_sweeps
    tune = autotune_group([(m, L) for (m, L, _, _, _) in specs], sweeps_per_call=8, reps=1)
    lats = [mcl.Lattice(m, L, sd) for (m, L, sd, _, _) in specs]
    betas = [b for (_, _, _, b, _) in specs]
    Ds = [d for (_, _, _, _, d) in specs]
    upd = float(sum(L * L for (_, L, _, _, _) in specs)) * n
    mcl.group_sweep(lats, [1] * len(lats), betas, Ds)           # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    mcl.group_sweep(lats, [n] * len(lats), betas, Ds)
    torch.cuda.synchronize()
    t_batched = time.perf_counter() - t0
    # the same call with one persistent launch per colour for every replica
    # (4 workgroups per CU walking the tile list) replayed from a captured
    # graph, whatever the tuner chose
    from paper_2502_18624_amd.autotune import get_tuning, set_tuning, tuning_dict, tuning_from_dict
    tuned = get_tuning()
    pg = tuning_from_dict(dict(tuning_dict(tuned), split_models=0, wg_per_cu=4, use_graph=1, graph_sweeps=32))
    set_tuning(pg)
    mcl.group_sweep(lats, [1] * len(lats), betas, Ds)           # warm-up
    mcl.group_sweep(lats, [1] * len(lats), betas, Ds)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    mcl.group_sweep(lats, [n] * len(lats), betas, Ds)           # a new shape: plain launches, then seen once
    mcl.group_sweep(lats, [n] * len(lats), betas, Ds)           # seen twice: captured and replayed
    torch.cuda.synchronize()
    t_pg = time.perf_counter() - t0
    set_tuning(tuned)
    t0 = time.perf_counter()
    for k in range(n):
        for lat, b, d in zip(lats, betas, Ds):
            lat.sweep(1, b, d)
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0
    for lat in lats:
        lat.free()
    return {"workload": "%d replicas (alternating Ising / Blume-Capel), L in {512..8192}, T ~ U[0.5,1.5] T_c, "
                        "D in {0,0.5,1}, %d sweeps each" % (len(specs), n),
            "spins": int(sum(L * L for (_, L, _, _, _) in specs)),
            "batched_updates_per_ns": round(upd / (t_batched * 1e9), 2),
            "plain_updates_per_ns": round(upd / (t_plain * 1e9), 2),
            "batched_over_plain": round(t_plain / t_batched, 3),
            "persistent_graph_updates_per_ns": round(2 * upd / (t_pg * 1e9), 2),
            "persistent_graph": "one launch per colour for all replicas, 4 workgroups per CU, 32-sweep graph "
                                "replays (two calls of %d sweeps; the second replays the captured graph)" % n,
            "tuning": {k: v for k, v in tune.items() if k != "rows_log2L"} | {
                "rows_by_L": {str(2 ** k): tune["rows_log2L"][k] for k in range(9, 14)}}}


def run_serving(args):
    """Poisson stream of quench jobs through the continuous-batching server:
    the first `serve_jobs` arrivals at 200 jobs/s (offered load far above one
    GPU), then `serve_sustainable_jobs` arrivals at about 70% of the rate the
    first trace measured."""
    from paper_2502_18624_amd.serve import Server, poisson_trace
    out = {}
    mean_work = None
    for name, rate, count in (("poisson_200_per_s", 200.0, args.serve_jobs),
                              ("sustainable", None, args.serve_sustainable_jobs)):
        if rate is None:
            cap = out["poisson_200_per_s"]["updates_per_ns"] * 1e9
            rate = 0.7 * cap / mean_work
        jobs = poisson_trace(count, rate_per_s=rate, seed=4)
        if mean_work is None:
            mean_work = sum(j.updates for j in jobs) / len(jobs)
        log("  serving %s: %d jobs at %.2f jobs/s" % (name, count, rate))
        # no result digests here: they copy each finished lattice to the host (a test aid)
        srv = Server(hbm_budget=250e9, tick_seconds=0.02, keep_digest=False)
        st = srv.run_trace(jobs)
        st["rate_per_s"] = round(rate, 3)
        st["arrival_window_s"] = round(max(j.arrival for j in jobs), 3)
        out[name] = {k: (round(v, 4) if isinstance(v, float) else v) for k, v in st.items()}
        log("  serving %s: p50 %.2f s, p99 %.2f s, %.1f updates/ns" % (
            name, st["latency_p50_s"], st["latency_p99_s"], st["updates_per_ns"]))
    out["workload"] = ("Poisson quench jobs (Ising/Blume-Capel 50/50), L = 64 round(2^U[10,15]/64), sweeps = "
                       "round(10^U[2,4]), T ~ U[0.5,1.5] T_c, D in {0,0.5,1}, admitted by footprint up to 250 GB; "
                       "first %d arrivals at 200 jobs/s, then %d at 70%% of the measured rate; one event per tick, "
                       "up to two ticks queued, retirement beside later ticks" % (
                           args.serve_jobs, args.serve_sustainable_jobs))
    return out


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

    from paper_2502_18624_amd.schedule import paper_times, pow2_times
    marks = paper_times(args.steps) if args.schedule == "paper" else pow2_times(args.steps)
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
            torch.cuda.synchronize()        # the measurement's time excludes the sweeps before it
            tm = time.perf_counter()
            out = lat.measure(mcl.CORR_PROTOCOL)
            t_meas += time.perf_counter() - tm
            cx, cy = mcl.correlation(out)
            c = 0.5 * (cx + cy)
            xi = mcl.correlation_length(out["r"], c, 1) if c[1] > 0 else None
            measures.append({"t": out["t"], "B": out["B"], "M": out["M"], "n_r": int(len(out["r"])),
                             "Cx1": int(out["Cx"][1]), "Cy1": int(out["Cy"][1]),
                             "schwinger_dyson": round(mcl.schwinger_dyson(out["sd"], beta), 7),
                             "xi12": round(xi, 3) if xi else None})
            log("  t=%d B=%d M=%d xi12=%s" % (out["t"], out["B"], out["M"], "%.2f" % xi if xi else "-"))
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    sweep_ms = sum(a.elapsed_time(b) for a, b, _ in ev)
    n_sweeps = sum(k for _, _, k in ev)
    assert n_sweeps == args.steps and lat.t == args.steps
    updates = float(L) * L * args.steps
    half_ms = sweep_ms / (2 * n_sweeps)
    half_updates = L * L / 2.0
    half_bytes = 3.0 * L * L / 4.0                 # read P_c, read P_{1-c}, write P_c (4-bit cells)
    hbm_gbs = half_bytes / (half_ms * 1e-3) / 1e9
    blocks_gps = half_updates / 4.0 / (half_ms * 1e-3) / 1e9   # one 32-bit draw per update
    traffic = measured_traffic("ising_4bit") if L == 2 ** 17 else None
    philox_alone = attainable_philox()
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
        "dtype": "u32",
        "arithmetic": "integer only: 4-bit cells packed in u32 words, u32 Philox4x32-10 draws, u32 thresholds",
        "data": "synthetic (seeded Philox4x32-10 random start)",
        "config": {"workload": "Ising quench, L=2^17, T=T_c, random +-1 start, %d sweeps, protocol C(r,t) and "
                               "B/M at %s, one lattice per launch" % (
                                   args.steps, "t=floor(2^(x/8)+0.5)" if args.schedule == "paper" else "t=2^k"),
                   "L": L, "seed": seed, "beta": beta, "measure_times": marks},
        "sweep_only_updates_per_ns": round(updates / (sweep_ms * 1e6), 2),
        "measure_share": round(t_meas / wall, 4),
        "measure_ms_avg": round(t_meas / len(measures) * 1e3, 3) if measures else None,
        "hbm_frac": round(hbm_gbs / HBM_PEAK_GBS, 4),
        "hbm_achieved_GBs": round(hbm_gbs, 1),
        "hbm_attainable_copy_GBs": attainable_copy(),
        "roofline": {"bound": "alu", "achieved": round(blocks_gps, 1), "peak": round(PHILOX_PEAK_GBLOCKS, 1),
                     "unit": "Gblocks/s", "frac": round(blocks_gps / PHILOX_PEAK_GBLOCKS, 4),
                     "traffic": traffic,
                     "traffic_source": traffic_source(),
                     "kernel": "half_sweep_kernel<Ising>", "avg_launch_ms": round(half_ms, 4),
                     "work_per_launch": "%d Philox4x32-10 blocks (one u32 draw per update), %d bytes" % (
                         int(half_updates / 4), int(half_bytes)),
                     "hbm_frac": round(hbm_gbs / HBM_PEAK_GBS, 4),
                     "valu_util_pmc": measured_valu_util("ising_4bit") if L == 2 ** 17 else None,
                     "philox_alone_Gblocks": philox_alone,
                     "frac_of_philox_alone": round(blocks_gps / philox_alone, 4) if philox_alone else None},
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
    ap.add_argument("--schedule", choices=("pow2", "paper"), default="pow2",
                    help="measurement times of the headline quench: t = 2^k, or the paper's floor(2^(x/8) + 0.5)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-full", action="store_true",
                    help="time the oracle on every workload of the plan (adds minutes of single-threaded sweeps)")
    ap.add_argument("--no-extras", action="store_true", help="only the Ising L=2^17 quench")
    ap.add_argument("--extras", default="bc,lut,batched,serving,scan",
                    help="comma list of the further legs: bc, lut, batched, serving, scan")
    ap.add_argument("--scan-updates", type=float, default=2e12, help="updates per size in the scan leg")
    ap.add_argument("--bc-sweeps", type=int, default=2000)
    ap.add_argument("--lut-sweeps", type=int, default=2000)
    ap.add_argument("--replicas", type=int, default=512)
    ap.add_argument("--batched-sweeps", type=int, default=100)
    ap.add_argument("--serve-jobs", type=int, default=300)
    ap.add_argument("--serve-sustainable-jobs", type=int, default=200)
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path (got --gpus %d)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)
    res = run(args)
    extras = [] if args.no_extras else [e for e in args.extras.split(",") if e]
    if "bc" in extras:
        log("bench: Blume-Capel L=2^16")
        res["blume_capel"] = run_blume_capel(args)
    if "lut" in extras:
        log("bench: Ising 1-bit L=2^17")
        res["ising_1bit"] = run_ising_1bit(args)
    if "batched" in extras:
        log("bench: batched vs plain")
        res["batched"] = run_batched(args)
        res["batched_over_plain"] = res["batched"]["batched_over_plain"]
    if "serving" in extras:
        log("bench: serving")
        res["serving"] = run_serving(args)
    if "scan" in extras:
        log("bench: throughput against L")
        res["scan"] = run_scan(args)
    if not args.no_cpu_baseline:
        log("bench: timing the CPU oracle sample")
        res["cpu_baseline"] = cpu_baseline(full=args.cpu_full)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
