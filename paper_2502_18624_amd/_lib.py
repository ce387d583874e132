"""ctypes binding of ``libmcl.so`` (the C ABI declared in ``include/mcl.h``).

Argument marshalling only: every step of the method runs in the library's
HIP kernels.  There is no CPU fallback; if the library is missing or cannot
be loaded, :func:`lib` raises.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmcl.so")

ISING, BC, ISING_LUT = 0, 1, 2
INIT_RANDOM, INIT_UP, INIT_DOWN, INIT_ZERO = 0, 1, 2, 3
CORR_NONE, CORR_FULL, CORR_PROTOCOL = 0, 1, 2

ERRORS = {
    0: "MCL_OK", -1: "MCL_EMODEL", -2: "MCL_EL", -3: "MCL_EBETA", -4: "MCL_ED",
    -5: "MCL_EINIT", -6: "MCL_ENOMEM", -7: "MCL_ERANGE", -8: "MCL_EHIP",
    -9: "MCL_EARG", -10: "MCL_EBUFSZ", -11: "MCL_ESPINS", -12: "MCL_ESCRATCH",
}


class MclError(RuntimeError):
    def __init__(self, code, where):
        self.code = code
        name = ERRORS.get(code, str(code))
        msg = "%s failed: %s (%s)" % (where, name, _strerror(code))
        if code == -8:
            msg += " [hip error %d]" % _lib_handle.mcl_last_hip_error()
        super().__init__(msg)


class MeasureOut(ctypes.Structure):
    _fields_ = [
        ("B", ctypes.c_int64), ("M", ctypes.c_int64), ("Q", ctypes.c_int64), ("t", ctypes.c_int64),
        ("counts", ctypes.c_int64 * 3), ("invalid", ctypes.c_int64),
        ("r", ctypes.POINTER(ctypes.c_int32)), ("Cx", ctypes.POINTER(ctypes.c_int64)),
        ("Cy", ctypes.POINTER(ctypes.c_int64)), ("nsrc", ctypes.POINTER(ctypes.c_int64)),
        ("r_cap", ctypes.c_int32), ("n_r", ctypes.c_int32), ("sd", ctypes.c_int64 * 9),
    ]


class GroupTuning(ctypes.Structure):
    _fields_ = [("rows_log2L", ctypes.c_int32 * 21), ("use_graph", ctypes.c_int32),
                ("largest_first", ctypes.c_int32), ("wg_per_cu", ctypes.c_int32),
                ("split_models", ctypes.c_int32), ("graph_sweeps", ctypes.c_int32)]


# Every entry point of include/mcl.h with its ctypes signature.
_P = ctypes.c_void_p
_I64, _U64, _I32, _U32, _INT, _DBL = (ctypes.c_int64, ctypes.c_uint64, ctypes.c_int32,
                                      ctypes.c_uint32, ctypes.c_int, ctypes.c_double)
SIGNATURES = {
    "mcl_query_bytes": (_INT, [_INT, _I64, ctypes.POINTER(_I64)]),
    "lattice_init": (_INT, [ctypes.POINTER(_P), _INT, _I64, _U64, _INT, _P, _I64, _P]),
    "sweep": (_INT, [_P, _I64, _DBL, _DBL]),
    "measure": (_INT, [_P, _INT, ctypes.POINTER(MeasureOut)]),
    "mcl_rset": (_INT, [_INT, _I64, _I64, ctypes.POINTER(_I32), _I32, ctypes.POINTER(_I32)]),
    "mcl_lut_table": (_INT, [_DBL, ctypes.POINTER(_U64)]),
    "mcl_thresholds": (_INT, [_INT, _DBL, _DBL, ctypes.POINTER(_U32), ctypes.POINTER(ctypes.c_uint8), _I32]),
    "lattice_read": (_INT, [_P, _P]),
    "lattice_read_window": (_INT, [_P, _I64, _I64, _I64, _I64, _P]),
    "lattice_read_packed": (_INT, [_P, _P, _I64]),
    "lattice_write_packed": (_INT, [_P, _P, _I64, _I64]),
    "lattice_write": (_INT, [_P, _P, _I64]),
    "lattice_info": (_INT, [_P, ctypes.POINTER(_INT), ctypes.POINTER(_I64), ctypes.POINTER(_U64),
                            ctypes.POINTER(_I64)]),
    "group_sweep": (_INT, [ctypes.POINTER(_P), _INT, ctypes.POINTER(_I64), ctypes.POINTER(_DBL),
                           ctypes.POINTER(_DBL)]),
    "group_sweep_noalloc": (_INT, [ctypes.POINTER(_P), _INT, ctypes.POINTER(_I64), ctypes.POINTER(_DBL),
                                   ctypes.POINTER(_DBL)]),
    "mcl_group_tuning_get": (_INT, [ctypes.POINTER(GroupTuning)]),
    "mcl_group_tuning_set": (_INT, [ctypes.POINTER(GroupTuning)]),
    "lattice_free": (_INT, [_P]),
    "mcl_strerror": (ctypes.c_char_p, [_INT]),
    "mcl_last_hip_error": (_INT, []),
}

_lib_handle = None


def lib():
    """Load ``libmcl.so`` (built in-tree by ``build.py``); raise if absent."""
    global _lib_handle
    if _lib_handle is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                "libmcl.so is not built (%s); run python paper_2502_18624_amd/build.py" % LIB_PATH)
        h = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(h, name)
            fn.restype = res
            fn.argtypes = args
        _lib_handle = h
    return _lib_handle


def _strerror(code):
    try:
        return lib().mcl_strerror(code).decode()
    except Exception:  # pragma: no cover - only reached while reporting another error
        return "?"


def check(code, where):
    if code < 0:
        raise MclError(code, where)
    return code
