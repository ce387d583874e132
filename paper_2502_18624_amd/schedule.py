"""Measurement times (section 3.3).

The paper measures at t = floor((2^{1/8})^x + 0.5) for positive integers x;
the benchmark workloads use its x = 0 (mod 8) members, t = 2^k."""
from __future__ import annotations

import math


def pow2_times(n_sweeps: int) -> list:
    """t = 1, 2, 4, ... <= n_sweeps."""
    out, t = [], 1
    while t <= n_sweeps:
        out.append(t)
        t <<= 1
    return out


def paper_times(n_sweeps: int) -> list:
    """Distinct floor(2^{x/8} + 0.5) <= n_sweeps for x = 1, 2, ..."""
    out, x = [], 1
    while True:
        t = int(math.floor(math.pow(2.0, x / 8.0) + 0.5))
        if t > n_sweeps:
            return out
        if not out or out[-1] != t:
            out.append(t)
        x += 1
