"""The measurement protocol of a quench (sections 1 and 3.3): a lattice
starts from its T = infinity sample, relaxes at (beta, D), and is measured
after t sweeps for t on a logarithmic schedule -- B, M, Q, E, the spin
counts, the Schwinger-Dyson value (eq. SDI) and C(r, t) along both axes.

    python -m paper_2502_18624_amd.quench --model ising --L 16384 --beta 0.4406868 \\
        --sweeps 1024 --schedule paper --out quench.jsonl

writes one JSON line per measurement time."""
from __future__ import annotations

import argparse
import json
import math
import sys

import numpy as np

from ._lib import BC, CORR_FULL, CORR_NONE, CORR_PROTOCOL, INIT_RANDOM, ISING, ISING_LUT
from .lattice import Lattice, correlation, correlation_length, energy, schwinger_dyson
from .schedule import paper_times, pow2_times

MODELS = {"ising": ISING, "blume-capel": BC, "bc": BC, "ising-1bit": ISING_LUT}
CORR = {"none": CORR_NONE, "full": CORR_FULL, "protocol": CORR_PROTOCOL}


def run_quench(model, L, seed, beta, D=0.0, sweeps=1024, schedule="pow2", corr=CORR_PROTOCOL, init=INIT_RANDOM,
               device="cuda", stream=None):
    """Yield one measurement dict per time of the schedule (t <= sweeps):
    the integer sums of measure(), plus "E", "schwinger_dyson" and, with a
    correlation mode, the normalised "Cx_norm" and "Cy_norm", the integral
    estimators "xi12" and "xi23" of the correlation length from their mean
    (None while it is not positive at r = 1), and "L_over_xi12", which
    section 1 wants to stay above about 50 for results free of finite-size
    effects."""
    times = paper_times(sweeps) if schedule == "paper" else pow2_times(sweeps)
    lat = Lattice(model, L, seed, init, device=device, stream=stream)
    try:
        for t in times:
            lat.sweep(t - lat.t, beta, D)
            m = lat.measure(corr)
            m["E"] = energy(m, D)
            m["schwinger_dyson"] = schwinger_dyson(m["sd"], beta) if math.isfinite(beta) else None
            if corr != CORR_NONE:
                m["Cx_norm"], m["Cy_norm"] = correlation(m)
                c = 0.5 * (m["Cx_norm"] + m["Cy_norm"])
                ok = c.size > 1 and c[1] > 0
                m["xi12"] = correlation_length(m["r"], c, 1) if ok else None
                m["xi23"] = correlation_length(m["r"], c, 2) if ok else None
                m["L_over_xi12"] = L / m["xi12"] if m["xi12"] else None
            yield m
    finally:
        lat.free()


def _jsonable(m):
    return {k: (v.tolist() if isinstance(v, np.ndarray) else v) for k, v in m.items()}


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--model", choices=sorted(MODELS), default="ising")
    ap.add_argument("--L", type=int, required=True)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--beta", type=float, required=True)
    ap.add_argument("--D", type=float, default=0.0)
    ap.add_argument("--sweeps", type=int, default=1024)
    ap.add_argument("--schedule", choices=("pow2", "paper"), default="pow2")
    ap.add_argument("--corr", choices=sorted(CORR), default="protocol")
    ap.add_argument("--out", default="-", help="JSON lines file, '-' for stdout")
    a = ap.parse_args(argv)
    out = sys.stdout if a.out == "-" else open(a.out, "w")
    try:
        for m in run_quench(MODELS[a.model], a.L, a.seed, a.beta, a.D, a.sweeps, a.schedule, CORR[a.corr]):
            out.write(json.dumps(_jsonable(m)) + "\n")
            out.flush()
    finally:
        if out is not sys.stdout:
            out.close()


if __name__ == "__main__":
    main()
