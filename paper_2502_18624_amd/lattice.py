"""Python face of the library: a :class:`Lattice` owns a torch device buffer
and a library handle; every call marshals arguments into the C ABI of
``include/mcl.h``.  PyTorch provides device memory and the stream only."""
from __future__ import annotations

import ctypes
import math

import numpy as np

from . import _lib
from ._lib import (BC, CORR_FULL, CORR_NONE, CORR_PROTOCOL, INIT_DOWN, INIT_RANDOM, INIT_UP,  # noqa: F401
                   INIT_ZERO, ISING, ISING_LUT, MeasureOut, check, lib)

_ALIGN = 256


def query_bytes(model: int, L: int) -> int:
    out = ctypes.c_int64()
    check(lib().mcl_query_bytes(model, L, ctypes.byref(out)), "mcl_query_bytes")
    return out.value


def rset(mode: int, L: int, t: int = 0) -> np.ndarray:
    need = ctypes.c_int32()
    rc = lib().mcl_rset(mode, L, t, None, 0, ctypes.byref(need))
    if rc not in (0, -10):
        check(rc, "mcl_rset")
    buf = np.zeros(max(need.value, 1), dtype=np.int32)
    n = check(lib().mcl_rset(mode, L, t, buf.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                             len(buf), ctypes.byref(need)), "mcl_rset")
    return buf[:n].copy()


def thresholds(model: int, beta: float, D: float = 0.0):
    """Ising: (T4, T8).  Blume-Capel: (thr[54], always[54])."""
    thr = np.zeros(54, dtype=np.uint32)
    alw = np.zeros(54, dtype=np.uint8)
    check(lib().mcl_thresholds(model, float(beta), float(D),
                               thr.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)),
                               alw.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)), 54), "mcl_thresholds")
    if model == ISING:
        return int(thr[0]), int(thr[1])
    return thr, alw.astype(bool)


def lut_table(beta: float):
    """The 16-entry table of the 1-bit mode (64-bit entries, up to 2^32)."""
    T = (ctypes.c_uint64 * 16)()
    check(lib().mcl_lut_table(float(beta), T), "mcl_lut_table")
    return [int(v) for v in T]


def schwinger_dyson(sd, beta: float) -> float:
    """Right-hand side of the Schwinger-Dyson identity (section 4, eq. SDI)
    from the histogram of measure()["sd"]: the site average of
    exp(-2 beta sigma h); 1 in equilibrium."""
    n = sum(int(v) for v in sd)
    if n == 0:
        raise ValueError("empty histogram")
    if not math.isfinite(beta) or beta < 0:
        raise ValueError("beta must be finite and non-negative")
    return math.fsum(int(v) * math.exp(-2.0 * beta * (k - 4)) for k, v in enumerate(sd) if v) / n


def energy(m: dict, D: float = 0.0) -> int | float:
    """E = -B + D Q from a measurement (J = 1; eq. IM for Ising, eq. BC)."""
    return -m["B"] + D * m["Q"] if D else -m["B"]


def correlation(m: dict):
    """Normalised correlations C_x(r) = S_x(r) / nsrc(r), C_y(r) likewise,
    from a measurement taken with a correlation mode (float64 arrays)."""
    ns = np.asarray(m["nsrc"], dtype=np.float64)
    return np.asarray(m["Cx"]) / ns, np.asarray(m["Cy"]) / ns


def correlation_length(r, C, k: int = 1) -> float:
    """Integral estimator xi_{k,k+1} = I_{k+1} / I_k of the correlation
    length xi(t), the growing domain size of a quench (section 1; the paper
    takes its estimators from a cited reference).  I_k is the integral of
    r^k C(r) dr over the measured distances r (ascending; the protocol's
    log-spaced tail included), by the trapezoid rule on that grid, up to the
    last distance before C first drops to zero or below (where noise takes
    over).  C is a normalised correlation, e.g. the mean of the two axes of
    correlation(m).  For C(r) = exp(-r/a), xi_{1,2} = 2a and xi_{2,3} = 3a."""
    r = np.asarray(r, dtype=np.float64)
    C = np.asarray(C, dtype=np.float64)
    if r.ndim != 1 or r.shape != C.shape or r.size < 2:
        raise ValueError("r and C must be 1-d arrays of the same length, at least 2")
    if np.any(np.diff(r) <= 0) or r[0] < 0:
        raise ValueError("r must be non-negative and strictly increasing")
    if k < 0:
        raise ValueError("k must be >= 0")
    nonpos = np.nonzero(C <= 0.0)[0]
    n = int(nonpos[0]) if nonpos.size else r.size
    if n < 2:
        raise ValueError("C must stay positive over at least two distances")
    r, C = r[:n], C[:n]

    def integral(p):
        f = r ** p * C
        return float(np.sum(0.5 * (f[1:] + f[:-1]) * np.diff(r)))

    return integral(k + 1) / integral(k)


class Lattice:
    """One L x L lattice resident in HBM (two 4-bit colour planes)."""

    def __init__(self, model: int, L: int, seed: int, init: int = INIT_RANDOM, device="cuda",
                 stream=None, mem=None):
        import torch

        self.model, self.L, self.seed = int(model), int(L), int(seed)
        self.nbytes = query_bytes(self.model, self.L)
        if mem is None:
            mem = torch.empty(self.nbytes + _ALIGN, dtype=torch.uint8, device=device)
        self.mem = mem
        base = mem.data_ptr()
        self.ptr = (base + _ALIGN - 1) // _ALIGN * _ALIGN
        if self.ptr + self.nbytes > base + mem.numel():
            raise ValueError("device buffer too small for L=%d" % L)
        self.stream = stream if stream is not None else torch.cuda.current_stream(mem.device)
        self._h = ctypes.c_void_p()
        check(lib().lattice_init(ctypes.byref(self._h), self.model, self.L, self.seed, int(init),
                                 ctypes.c_void_p(self.ptr), self.nbytes,
                                 ctypes.c_void_p(self.stream.cuda_stream)), "lattice_init")

    # -- state -----------------------------------------------------------
    @property
    def handle(self):
        return self._h

    @property
    def t(self) -> int:
        t = ctypes.c_int64()
        check(lib().lattice_info(self._h, None, None, None, ctypes.byref(t)), "lattice_info")
        return t.value

    # -- the method ------------------------------------------------------
    def sweep(self, n: int, beta: float, D: float = 0.0) -> None:
        check(lib().sweep(self._h, int(n), float(beta), float(D)), "sweep")

    def measure(self, corr: int = CORR_NONE) -> dict:
        out = MeasureOut()
        cap = 0
        if corr != CORR_NONE:
            cap = len(rset(corr, self.L, self.t))
        r = np.zeros(max(cap, 1), dtype=np.int32)
        cx = np.zeros(max(cap, 1), dtype=np.int64)
        cy = np.zeros(max(cap, 1), dtype=np.int64)
        ns = np.zeros(max(cap, 1), dtype=np.int64)
        out.r = r.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
        out.Cx = cx.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
        out.Cy = cy.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
        out.nsrc = ns.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
        out.r_cap = cap
        check(lib().measure(self._h, int(corr), ctypes.byref(out)), "measure")
        n = out.n_r
        return {"B": out.B, "M": out.M, "Q": out.Q, "t": out.t, "counts": list(out.counts),
                "invalid": out.invalid, "r": r[:n].copy(), "Cx": cx[:n].copy(), "Cy": cy[:n].copy(),
                "nsrc": ns[:n].copy(), "sd": list(out.sd)}

    # -- host copies (parity checks, checkpoints) -------------------------
    def read(self) -> np.ndarray:
        s = np.empty((self.L, self.L), dtype=np.int8)
        check(lib().lattice_read(self._h, s.ctypes.data_as(ctypes.c_void_p)), "lattice_read")
        return s

    def read_window(self, x0: int, y0: int, w: int, h: int) -> np.ndarray:
        s = np.empty((h, w), dtype=np.int8)
        check(lib().lattice_read_window(self._h, x0, y0, w, h, s.ctypes.data_as(ctypes.c_void_p)),
              "lattice_read_window")
        return s

    def write(self, spins: np.ndarray, t: int) -> None:
        s = np.ascontiguousarray(spins, dtype=np.int8)
        if s.shape != (self.L, self.L):
            raise ValueError("expected shape (%d, %d)" % (self.L, self.L))
        check(lib().lattice_write(self._h, s.ctypes.data_as(ctypes.c_void_p), int(t)), "lattice_write")

    def read_packed(self) -> np.ndarray:
        bits = 1 if self.model == ISING_LUT else 4
        buf = np.empty(self.L * self.L * bits // 8, dtype=np.uint8)
        check(lib().lattice_read_packed(self._h, buf.ctypes.data_as(ctypes.c_void_p), buf.nbytes),
              "lattice_read_packed")
        return buf

    def write_packed(self, buf: np.ndarray, t: int) -> None:
        b = np.ascontiguousarray(buf, dtype=np.uint8)
        check(lib().lattice_write_packed(self._h, b.ctypes.data_as(ctypes.c_void_p), b.nbytes, int(t)),
              "lattice_write_packed")

    def free(self) -> None:
        if self._h:
            lib().lattice_free(self._h)
            self._h = ctypes.c_void_p()
            self.mem = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def group_sweep(lattices, n, beta, D=None, noalloc=False) -> None:
    """Batched path: advance each lattice i by n[i] sweeps at (beta[i], D[i]).
    With noalloc, the call goes through group_sweep_noalloc (fixed
    workspaces, plain launches, no allocation)."""
    k = len(lattices)
    n = list(n) if np.ndim(n) else [int(n)] * k
    beta = list(beta) if np.ndim(beta) else [float(beta)] * k
    D = [0.0] * k if D is None else (list(D) if np.ndim(D) else [float(D)] * k)
    hs = (ctypes.c_void_p * k)(*[l.handle.value for l in lattices])
    nn = (ctypes.c_int64 * k)(*[int(v) for v in n])
    bb = (ctypes.c_double * k)(*[float(v) for v in beta])
    dd = (ctypes.c_double * k)(*[float(v) for v in D])
    if noalloc:
        check(lib().group_sweep_noalloc(hs, k, nn, bb, dd), "group_sweep_noalloc")
    else:
        check(lib().group_sweep(hs, k, nn, bb, dd), "group_sweep")
