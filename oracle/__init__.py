"""CPU oracle (ctypes wrapper around ``oracle.c``).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's
CPU-baseline leg may import this module; the product package never does, and
this module never imports the product package.  See ``oracle.h`` for what each
routine computes and which passage of the paper it follows.

The lattice is a NumPy ``int8`` array of shape ``(L, L)`` indexed ``[y, x]``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

ISING, BC, ISING_LUT = 0, 1, 2
INIT_RANDOM, INIT_UP, INIT_DOWN, INIT_ZERO = 0, 1, 2, 3
CORR_FULL, CORR_PROTOCOL = 1, 2


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain -O2, OpenMP for the row split)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-std=c99", "-O2", "-fopenmp", "-fPIC", "-shared",
               "-Wall", "-Wextra", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        L = ctypes.CDLL(_LIB)
        u32, u64, i64, i32 = ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int64, ctypes.c_int32
        P = ctypes.POINTER
        L.ora_philox4x32_10.argtypes = [P(u32), P(u32), P(u32)]
        L.ora_accept_draw.argtypes = [u64, u32, ctypes.c_int, u64]
        L.ora_accept_draw.restype = u32
        L.ora_proposal_bit.argtypes = [u64, u32, ctypes.c_int, u64]
        L.ora_proposal_bit.restype = ctypes.c_int
        L.ora_init_draw.argtypes = [u64, u64]
        L.ora_init_draw.restype = u32
        L.ora_lut_table.argtypes = [ctypes.c_double, P(u64)]
        L.ora_lut_lookup.argtypes = [P(u64), u32]
        L.ora_lut_lookup.restype = ctypes.c_int
        L.ora_lut_draw.argtypes = [u64, u32, ctypes.c_int, ctypes.c_int, u64]
        L.ora_lut_draw.restype = u32
        L.ora_threshold.argtypes = [ctypes.c_double, ctypes.c_double]
        L.ora_threshold.restype = u32
        L.ora_ising_flip_prob.argtypes = [ctypes.c_int, ctypes.c_double]
        L.ora_ising_flip_prob.restype = ctypes.c_double
        L.ora_bc_accept_prob.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                         ctypes.c_double, ctypes.c_double]
        L.ora_bc_accept_prob.restype = ctypes.c_double
        L.ora_init.argtypes = [ctypes.c_void_p, ctypes.c_int, i64, u64, ctypes.c_int]
        L.ora_init.restype = ctypes.c_int
        L.ora_sweep.argtypes = [ctypes.c_void_p, ctypes.c_int, i64, u64, i64, i64,
                                ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                P(i64), P(i64)]
        L.ora_sweep.restype = ctypes.c_int
        L.ora_measure.argtypes = [ctypes.c_void_p, i64, P(i64), P(i64), P(i64), P(i64), ctypes.c_int]
        L.ora_rset.argtypes = [ctypes.c_int, i64, i64, P(i32), ctypes.c_int]
        L.ora_rset.restype = ctypes.c_int
        L.ora_rc.argtypes = [i64, i64]
        L.ora_rc.restype = i64
        L.ora_g.argtypes = [i64]
        L.ora_g.restype = ctypes.c_double
        L.ora_corr.argtypes = [ctypes.c_void_p, i64, ctypes.c_int, P(i32), ctypes.c_int,
                               P(i64), P(i64), P(i64), ctypes.c_int]
        L.ora_sd_hist.argtypes = [ctypes.c_void_p, i64, P(i64), ctypes.c_int]
        L.ora_init_window.argtypes = [ctypes.c_void_p, i64, i64, i64, ctypes.c_int, i64, u64, ctypes.c_int]
        L.ora_init_window.restype = ctypes.c_int
        L.ora_sweep_window.argtypes = [ctypes.c_void_p, i64, i64, i64, ctypes.c_int, i64, u64, i64, i64,
                                       ctypes.c_double, ctypes.c_double]
        L.ora_sweep_window.restype = ctypes.c_int
        L.ora_series.argtypes = [ctypes.c_void_p, ctypes.c_int, i64, u64, i64, i64,
                                 ctypes.c_double, ctypes.c_double, P(i64), P(i64), P(i64)]
        L.ora_series.restype = ctypes.c_int
        _lib = L
    return _lib


def _ptr(a, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct))


def philox(ctr, key):
    c = (ctypes.c_uint32 * 4)(*[int(v) & 0xFFFFFFFF for v in ctr])
    k = (ctypes.c_uint32 * 2)(*[int(v) & 0xFFFFFFFF for v in key])
    o = (ctypes.c_uint32 * 4)()
    lib().ora_philox4x32_10(c, k, o)
    return [int(v) for v in o]


def accept_draw(seed, t, color, k):
    return int(lib().ora_accept_draw(seed, t, color, k))


def proposal_bit(seed, t, color, k):
    return int(lib().ora_proposal_bit(seed, t, color, k))


def init_draw(seed, n):
    return int(lib().ora_init_draw(seed, n))


def lut_table(beta):
    T = (ctypes.c_uint64 * 16)()
    lib().ora_lut_table(float(beta), T)
    return [int(v) for v in T]


def lut_lookup(T, u):
    arr = (ctypes.c_uint64 * 16)(*T)
    return int(lib().ora_lut_lookup(arr, u))


def lut_draw(seed, t, color, e, g):
    return int(lib().ora_lut_draw(seed, t, color, e, g))


def threshold(beta, dE):
    return int(lib().ora_threshold(float(beta), float(dE)))


def ising_thresholds(beta):
    return threshold(beta, 4.0), threshold(beta, 8.0)


def ising_flip_prob(aligned, beta):
    return float(lib().ora_ising_flip_prob(int(aligned), float(beta)))


def bc_accept_prob(s, h, b, beta, D):
    return float(lib().ora_bc_accept_prob(int(s), int(h), int(b), float(beta), float(D)))


def bc_table(beta, D):
    """(thr, always) arrays of shape (3, 2, 9) indexed [s+1, b, h+4]."""
    thr = np.zeros((3, 2, 9), dtype=np.uint64)
    always = np.zeros((3, 2, 9), dtype=bool)
    for si in range(3):
        for b in range(2):
            for hi in range(9):
                p = bc_accept_prob(si - 1, hi - 4, b, beta, D)
                s, h = si - 1, hi - 4
                s2 = ((si + 1 + b) % 3) - 1
                dE = float(-h * (s2 - s)) + D * float(s2 * s2 - s * s)
                if dE <= 0.0:
                    always[si, b, hi] = True
                else:
                    thr[si, b, hi] = threshold(beta, dE)
                    assert p == thr[si, b, hi] / 2.0 ** 32
    return thr, always


def init(model, L, seed, init_state=INIT_RANDOM):
    s = np.empty((L, L), dtype=np.int8)
    rc = lib().ora_init(s.ctypes.data, model, L, seed, init_state)
    if rc:
        raise ValueError("ora_init failed (%d)" % rc)
    return s


def sweep(s, model, seed, t0, n, beta, D=0.0, nthreads=1, track=False):
    """Advance ``s`` in place by ``n`` sweeps starting at sweep index ``t0``."""
    assert s.dtype == np.int8 and s.flags.c_contiguous and s.shape[0] == s.shape[1]
    L = s.shape[0]
    dB = ctypes.c_int64(0)
    dQ = ctypes.c_int64(0)
    rc = lib().ora_sweep(s.ctypes.data, model, L, seed, t0, n, float(beta), float(D),
                         nthreads, ctypes.byref(dB), ctypes.byref(dQ))
    if rc:
        raise ValueError("ora_sweep failed (%d)" % rc)
    if track:
        return dB.value, dQ.value
    return None


def measure(s, nthreads=1):
    L = s.shape[0]
    B, M, Q = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    cnt = (ctypes.c_int64 * 3)()
    lib().ora_measure(s.ctypes.data, L, ctypes.byref(B), ctypes.byref(M), ctypes.byref(Q), cnt, int(nthreads))
    return {"B": B.value, "M": M.value, "Q": Q.value, "counts": [int(c) for c in cnt]}


def g(L):
    return float(lib().ora_g(L))


def rc(L, t):
    return int(lib().ora_rc(L, t))


def rset(mode, L, t=0):
    cap = 16
    while True:
        buf = np.zeros(cap, dtype=np.int32)
        n = lib().ora_rset(mode, L, t, _ptr(buf, ctypes.c_int32), cap)
        if n >= 0:
            return buf[:n].copy()
        cap = -n


def corr(s, mode, r, nthreads=1):
    L = s.shape[0]
    r = np.ascontiguousarray(r, dtype=np.int32)
    nr = len(r)
    Cx = np.zeros(nr, dtype=np.int64)
    Cy = np.zeros(nr, dtype=np.int64)
    ns = np.zeros(nr, dtype=np.int64)
    lib().ora_corr(s.ctypes.data, L, mode, _ptr(r, ctypes.c_int32), nr,
                   _ptr(Cx, ctypes.c_int64), _ptr(Cy, ctypes.c_int64), _ptr(ns, ctypes.c_int64), int(nthreads))
    return Cx, Cy, ns


def sd_hist(s, nthreads=1):
    h = np.zeros(9, dtype=np.int64)
    lib().ora_sd_hist(s.ctypes.data, s.shape[0], _ptr(h, ctypes.c_int64), int(nthreads))
    return h


def window_run(model, L, seed, x0, y0, P, n, beta, D=0.0, init_state=INIT_RANDOM, t0=0):
    """Patch of P x P sites at (x0, y0) of an L x L lattice after n sweeps
    from its initial state; rows and columns at least 2n from the patch edge
    are exact (light cone)."""
    p = np.empty((P, P), dtype=np.int8)
    rc = lib().ora_init_window(p.ctypes.data, P, x0, y0, model, L, seed, init_state)
    if rc:
        raise ValueError("ora_init_window failed (%d)" % rc)
    rc = lib().ora_sweep_window(p.ctypes.data, P, x0, y0, model, L, seed, t0, n, float(beta), float(D))
    if rc:
        raise ValueError("ora_sweep_window failed (%d)" % rc)
    return p


def series(s, model, seed, t0, n, beta, D=0.0):
    L = s.shape[0]
    Bs = np.zeros(n, dtype=np.int64)
    Ms = np.zeros(n, dtype=np.int64)
    Qs = np.zeros(n, dtype=np.int64)
    rcode = lib().ora_series(s.ctypes.data, model, L, seed, t0, n, float(beta), float(D),
                             _ptr(Bs, ctypes.c_int64), _ptr(Ms, ctypes.c_int64),
                             _ptr(Qs, ctypes.c_int64))
    if rcode:
        raise ValueError("ora_series failed (%d)" % rcode)
    return Bs, Ms, Qs


def schedule_pow2(n_sweeps):
    """Measurement times t = 2^k <= n_sweeps (the x = 0 mod 8 members of the
    log-spaced schedule of section 3.3)."""
    out, t = [], 1
    while t <= n_sweeps:
        out.append(t)
        t *= 2
    return out


def schedule_paper(n_sweeps):
    """Distinct t = floor((2^{1/8})^x + 0.5) <= n_sweeps, x = 1, 2, ...
    (section 3.3)."""
    out, x = [], 1
    while True:
        t = int(np.floor(2.0 ** (x / 8.0) + 0.5))
        if t > n_sweeps:
            break
        if not out or out[-1] != t:
            out.append(t)
        x += 1
    return out
