"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every function ``include/mcl.h`` declares, validates arguments before any
device work, and its host tables (thresholds, correlation distances) equal
the oracle's, which were built independently."""
import ctypes
import math
import os
import re
import subprocess

import numpy as np
import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mcl.h")
BETA_C = math.log(1 + math.sqrt(2)) / 2


@pytest.fixture(scope="module")
def mcl():
    import paper_2502_18624_amd as m
    return m


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*([a-z_][a-z_0-9]*)\s*\(", src, flags=re.M)
    return sorted(set(n for n in names if n not in ("if", "while")))


def test_header_declares_the_entry_points():
    names = declared_functions()
    for must in ("lattice_init", "sweep", "measure", "group_sweep", "lattice_read", "lattice_write",
                 "lattice_free", "mcl_query_bytes", "mcl_strerror"):
        assert must in names


def test_library_exports_every_declared_symbol(mcl):
    lib = mcl.lib()
    out = subprocess.run(["nm", "-D", "--defined-only", lib._name], capture_output=True, text=True, check=True)
    exported = set(line.split()[-1] for line in out.stdout.splitlines() if line.strip())
    for name in declared_functions():
        assert name in exported, name
        assert getattr(lib, name) is not None
    # the python binding declares a signature for each of them
    from paper_2502_18624_amd._lib import SIGNATURES
    assert set(declared_functions()) == set(SIGNATURES)


def test_library_does_not_link_the_oracle(mcl):
    out = subprocess.run(["nm", "-D", mcl.lib()._name], capture_output=True, text=True, check=True)
    assert "ora_" not in out.stdout
    deps = subprocess.run(["ldd", mcl.lib()._name], capture_output=True, text=True).stdout
    assert "oracle" not in deps


def test_query_bytes(mcl):
    assert mcl.query_bytes(mcl.ISING, 256) >= 256 * 256 // 2
    assert mcl.query_bytes(mcl.ISING, 2**17) >= 2**33
    for L in (64, 256, 2**16, 2**17):
        # two 4-bit planes, then scratch: the sampled columns as two bit planes
        # (L^2 / 128 bytes each, at least 4 bytes a row) + O(L) sums
        assert L * L // 2 <= mcl.query_bytes(mcl.BC, L) <= L * L // 2 + max(L * L // 64, 8 * L) + 64 * L + 8192
    with pytest.raises(mcl.MclError):
        mcl.query_bytes(mcl.ISING, 96 + 1)
    with pytest.raises(mcl.MclError):
        mcl.query_bytes(7, 256)
    with pytest.raises(mcl.MclError):
        mcl.query_bytes(mcl.ISING, 32)


def test_query_bytes_one_bit(mcl):
    for L in (256, 768, 2**16, 2**17):
        # two 1-bit planes, one bit plane of the sampled columns, O(L) sums and the 32 KiB bucket table
        assert L * L // 8 + 32768 <= mcl.query_bytes(mcl.ISING_LUT, L) <= L * L // 8 + max(L * L // 128, 4 * L) + 64 * L + 8192 + 32768
    for L in (64, 128, 320):                    # a row of a 1-bit plane is whole 16-byte vectors
        with pytest.raises(mcl.MclError):
            mcl.query_bytes(mcl.ISING_LUT, L)


@pytest.mark.parametrize("beta", [0.0, 0.05, 0.3, BETA_C, BETA_C / 0.9, BETA_C / 0.5, 3.0, 6.0, float("inf")])
def test_lut_table_equals_oracle(mcl, beta):
    assert mcl.lut_table(beta) == oracle.lut_table(beta)


@pytest.mark.parametrize("beta", [0.0, 0.1, BETA_C, BETA_C / 0.9, BETA_C / 0.5, 3.0, float("inf")])
def test_ising_thresholds_equal_oracle(mcl, beta):
    assert mcl.thresholds(mcl.ISING, beta) == oracle.ising_thresholds(beta)


@pytest.mark.parametrize("beta,D", [(1 / 1.4, 1.0), (0.3, 0.0), (0.6, 0.5), (1.0, -3.0), (2.0, 2.7),
                                    (float("inf"), 1.0), (0.0, 1.0)])
def test_bc_table_equals_oracle(mcl, beta, D):
    thr, alw = mcl.thresholds(mcl.BC, beta, D)
    othr, oalw = oracle.bc_table(beta, D)
    assert np.array_equal(thr.reshape(3, 2, 9).astype(np.uint64), othr)
    assert np.array_equal(alw.reshape(3, 2, 9), oalw)


@pytest.mark.parametrize("L", [64, 128, 256, 1024, 2**15, 2**16, 2**17, 2**18])
@pytest.mark.parametrize("t", [0, 1, 2, 1000, 1024, 2000, 2048, 10**5])
def test_protocol_distances_equal_oracle(mcl, L, t):
    assert np.array_equal(mcl.rset(mcl.CORR_PROTOCOL, L, t), oracle.rset(oracle.CORR_PROTOCOL, L, t))


@pytest.mark.parametrize("L", [64, 192, 256, 4096])
def test_full_distances_equal_oracle(mcl, L):
    assert np.array_equal(mcl.rset(mcl.CORR_FULL, L), oracle.rset(oracle.CORR_FULL, L))


def test_argument_errors_before_device_work(mcl):
    lib = mcl.lib()
    h = ctypes.c_void_p()
    fake = ctypes.c_void_p(1 << 20)     # never dereferenced: every call below fails validation first
    nb = mcl.query_bytes(mcl.ISING, 256)
    assert lib.lattice_init(ctypes.byref(h), 5, 256, 1, 0, fake, nb, None) == -1          # MCL_EMODEL
    assert lib.lattice_init(ctypes.byref(h), 0, 100, 1, 0, fake, nb, None) == -2          # MCL_EL
    assert lib.lattice_init(ctypes.byref(h), 0, 256, 1, 3, fake, nb, None) == -5          # ZERO with Ising
    assert lib.lattice_init(ctypes.byref(h), 0, 256, 1, 9, fake, nb, None) == -5
    assert lib.lattice_init(ctypes.byref(h), 2, 320, 1, 0, fake, nb, None) == -2          # 1-bit: L % 256
    assert lib.lattice_init(ctypes.byref(h), 2, 256, 1, 3, fake, nb, None) == -5          # ZERO, 1-bit Ising
    assert lib.mcl_lut_table(float("nan"), (ctypes.c_uint64 * 16)()) == -3
    assert lib.mcl_lut_table(-0.5, (ctypes.c_uint64 * 16)()) == -3
    assert lib.mcl_lut_table(0.5, None) == -9
    assert lib.lattice_init(ctypes.byref(h), 0, 256, 1, 0, fake, nb - 1, None) == -6     # MCL_ENOMEM
    assert lib.lattice_init(ctypes.byref(h), 0, 256, 1, 0, None, nb, None) == -9          # MCL_EARG
    assert lib.sweep(None, 1, 0.4, 0.0) == -9
    assert lib.measure(None, 0, None) == -9
    assert lib.group_sweep(None, -1, None, None, None) == -9
    assert lib.mcl_rset(2, 96 * 2, 0, None, 0, None) == -2                               # protocol needs 2^k
    assert lib.mcl_thresholds(0, float("nan"), 0.0, (ctypes.c_uint32 * 54)(), None, 54) == -3
    assert lib.mcl_thresholds(0, -1.0, 0.0, (ctypes.c_uint32 * 54)(), None, 54) == -3
    for D in (float("nan"), float("inf"), -float("inf")):                               # MCL_ED
        assert lib.mcl_thresholds(1, 0.5, D, (ctypes.c_uint32 * 54)(), (ctypes.c_uint8 * 54)(), 54) == -4
    for code in range(0, -12, -1):
        assert lib.mcl_strerror(code)


def test_group_tuning_roundtrip_and_validation(mcl):
    from paper_2502_18624_amd._lib import GroupTuning
    lib = mcl.lib()
    saved = GroupTuning()
    assert lib.mcl_group_tuning_get(ctypes.byref(saved)) == 0
    assert all(r in (8, 16, 32, 64) for r in saved.rows_log2L)
    t = GroupTuning()
    ctypes.memmove(ctypes.byref(t), ctypes.byref(saved), ctypes.sizeof(t))
    t.rows_log2L[10] = 12                     # not a supported band height
    assert lib.mcl_group_tuning_set(ctypes.byref(t)) == -9
    t.rows_log2L[10] = 64
    for field, bad in (("wg_per_cu", -1), ("wg_per_cu", 33), ("split_models", 2), ("graph_sweeps", 0),
                       ("graph_sweeps", 65), ("use_graph", 2), ("largest_first", -1)):
        good = getattr(t, field)
        setattr(t, field, bad)
        assert lib.mcl_group_tuning_set(ctypes.byref(t)) == -9, field
        setattr(t, field, good)
    t.use_graph, t.wg_per_cu, t.split_models, t.graph_sweeps = 1, 4, 1, 16
    assert lib.mcl_group_tuning_set(ctypes.byref(t)) == 0
    back = GroupTuning()
    lib.mcl_group_tuning_get(ctypes.byref(back))
    assert back.rows_log2L[10] == 64 and back.use_graph == 1
    assert (back.wg_per_cu, back.split_models, back.graph_sweeps) == (4, 1, 16)
    assert lib.mcl_group_tuning_set(ctypes.byref(saved)) == 0
    assert lib.group_sweep(None, 0, None, None, None) == 0     # empty group is a no-op


@pytest.mark.parametrize("model,beta", [(0, 0.3), (0, BETA_C), (1, 0.7), (2, 1.1)])
def test_schwinger_dyson_helper_equals_site_average(mcl, model, beta):
    """Right-hand side of eq. SDI from the 9-bin histogram equals the site
    average of exp(-2 beta sigma h) written out over the lattice."""
    s = oracle.init(model, 64, 17)
    oracle.sweep(s, model, 17, 0, 5, beta, 0.5)
    h = np.roll(s, 1, 0) + np.roll(s, -1, 0) + np.roll(s, 1, 1) + np.roll(s, -1, 1)
    direct = float(np.mean(np.exp(-2.0 * beta * s.astype(np.float64) * h)))
    assert mcl.schwinger_dyson(oracle.sd_hist(s), beta) == pytest.approx(direct, rel=1e-13)
    up = np.ones((64, 64), dtype=np.int8)
    assert mcl.schwinger_dyson(oracle.sd_hist(up), beta) == pytest.approx(math.exp(-8 * beta), rel=1e-15)
    with pytest.raises(ValueError):
        mcl.schwinger_dyson([0] * 9, beta)


def test_header_is_plain_c_and_cpp(tmp_path):
    """include/mcl.h compiles as strict C99 and as C++ (no torch or HIP types
    in its signatures)."""
    src = tmp_path / "h.c"
    src.write_text('#include "mcl.h"\nint main(void) { mcl_measure_out o = {0}; return (int)o.n_r; }\n')
    inc = os.path.join(ROOT, "include")
    subprocess.run(["gcc", "-std=c99", "-Wall", "-Wextra", "-Werror", "-fsyntax-only", "-I", inc, str(src)],
                   check=True)
    subprocess.run(["g++", "-x", "c++", "-Wall", "-Werror", "-fsyntax-only", "-I", inc, str(src)], check=True)


def test_c_program_builds_against_the_abi(mcl, tmp_path):
    from tests import c_abi
    assert os.path.exists(c_abi.build(str(tmp_path / "q")))
