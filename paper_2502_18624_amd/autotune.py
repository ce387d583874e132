"""Autotuner of the batched path.

The tunables of ``group_sweep`` -- band height per lattice size, the
persistent grid (workgroups per compute unit, or one per tile), one launch
per colour for every model or one per model, hipGraph replay, tile order --
change how the work is laid on the chip, never what it computes: the draws
are keyed by the logical site.  The tuner
therefore times candidates on scratch lattices with the same (model, L) mix
as the real group (same shapes, their own seeds), leaves the real lattices
untouched, and installs the fastest setting process-wide.  Results are
cached per (device, shape mix, sweeps per call)."""
from __future__ import annotations

import ctypes
import json
import os
import time
from collections import Counter

from ._lib import GroupTuning, check, lib

ROWS = (8, 16, 32, 64)
_cache = {}


def get_tuning() -> GroupTuning:
    t = GroupTuning()
    check(lib().mcl_group_tuning_get(ctypes.byref(t)), "mcl_group_tuning_get")
    return t


def set_tuning(t: GroupTuning) -> None:
    check(lib().mcl_group_tuning_set(ctypes.byref(t)), "mcl_group_tuning_set")


FIELDS = ("use_graph", "largest_first", "wg_per_cu", "split_models", "graph_sweeps")
# candidate values of the scalar fields, searched after the band heights
CHOICES = {"wg_per_cu": (0, 2, 4, 8), "split_models": (0, 1), "use_graph": (0, 1), "largest_first": (0, 1)}


def tuning_dict(t: GroupTuning) -> dict:
    d = {"rows_log2L": list(t.rows_log2L)}
    for f in FIELDS:
        d[f] = int(getattr(t, f))
    return d


def tuning_from_dict(d: dict) -> GroupTuning:
    t = get_tuning()
    for k, v in enumerate(d["rows_log2L"]):
        t.rows_log2L[k] = int(v)
    for f in FIELDS:
        if f in d:
            setattr(t, f, int(d[f]))
    return t


def _log2(L: int) -> int:
    return int(L).bit_length() - 1


def _time_group(lats, n, betas, Ds, reps):
    import torch

    from .lattice import group_sweep
    group_sweep(lats, [n] * len(lats), betas, Ds)          # warm-up (and graph capture)
    torch.cuda.synchronize()
    best = float("inf")
    for _ in range(reps):
        t0 = time.perf_counter()
        group_sweep(lats, [n] * len(lats), betas, Ds)
        torch.cuda.synchronize()
        best = min(best, time.perf_counter() - t0)
    return best


def autotune_group(shapes, sweeps_per_call=8, reps=2, beta=0.44, D=0.5, verbose=False, cache_file=None) -> dict:
    """shapes: iterable of (model, L).  Returns the chosen tuning (as a dict)
    after installing it."""
    import torch

    from .lattice import Lattice

    mix = sorted(Counter((int(m), int(L)) for m, L in shapes).items())
    key = json.dumps([torch.cuda.get_device_name(), mix, int(sweeps_per_call)])
    if cache_file and not _cache and os.path.exists(cache_file):
        try:
            with open(cache_file) as f:
                _cache.update(json.load(f))
        except (OSError, ValueError):
            pass
    if key in _cache:
        set_tuning(tuning_from_dict(_cache[key]))
        return _cache[key]
    lats = []
    for i, ((m, L), c) in enumerate(mix):
        for j in range(c):
            lats.append(Lattice(m, L, 900000 + 1000 * i + j))
    betas = [beta] * len(lats)
    Ds = [D] * len(lats)
    cur = get_tuning()
    best_t = _time_group(lats, sweeps_per_call, betas, Ds, reps)
    buckets = sorted(set(_log2(L) for (_, L), _ in mix))
    # coordinate search: band height per size bucket, then graph, then order
    for b in buckets:
        for r in ROWS:
            if r == cur.rows_log2L[b]:
                continue
            cand = tuning_from_dict(tuning_dict(cur))
            cand.rows_log2L[b] = r
            set_tuning(cand)
            el = _time_group(lats, sweeps_per_call, betas, Ds, reps)
            if verbose:
                print("  rows[2^%d]=%d: %.3f ms" % (b, r, el * 1e3))
            if el < best_t:
                best_t, cur = el, cand
    for field, values in CHOICES.items():
        for v in values:
            if v == getattr(cur, field):
                continue
            cand = tuning_from_dict(tuning_dict(cur))
            setattr(cand, field, v)
            set_tuning(cand)
            el = _time_group(lats, sweeps_per_call, betas, Ds, reps)
            if verbose:
                print("  %s=%d: %.3f ms" % (field, v, el * 1e3))
            if el < best_t:
                best_t, cur = el, cand
    set_tuning(cur)
    for l in lats:
        l.free()
    res = tuning_dict(cur)
    res["seconds_per_call"] = best_t
    _cache[key] = res
    if cache_file:
        try:
            with open(cache_file, "w") as f:
                json.dump(_cache, f)
        except OSError:
            pass
    return res
