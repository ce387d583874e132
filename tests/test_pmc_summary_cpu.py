"""The PMC summariser (paper_2502_18624_amd.pmc_summary) on synthetic
rocprofv3 counter files: the copy kernel's known 4 GiB in / 4 GiB out set
the FETCH_SIZE / WRITE_SIZE scales, which turn a sweep kernel's counters
into bytes per launch; the VALU figures follow their definitions.  CPU only."""
import csv

import pytest

from paper_2502_18624_amd import pmc_summary

ISING = "void mcl::(anonymous namespace)::half_sweep_kernel<0, true, %d>(unsigned int*, unsigned int const*, " \
        "unsigned int, unsigned int, unsigned int, unsigned int const*, unsigned int, unsigned int, unsigned int, " \
        "unsigned int, mcl::BCTable)"
COPY = "copy_kernel(HIP_vector_type<unsigned int, 4u> const*, HIP_vector_type<unsigned int, 4u>*, long)"


def _write(path, rows):
    path.parent.mkdir(parents=True, exist_ok=True)
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for name, counter, value in rows:
            w.writerow({"Kernel_Name": name, "Counter_Name": counter, "Counter_Value": value})


def test_kernel_names_are_shortened():
    assert pmc_summary.short(ISING % 1) == "half_sweep_kernel<0, true, 1>"
    assert pmc_summary.short(COPY) == "copy_kernel"
    assert pmc_summary.short("__amd_rocclr_copyBuffer") == "__amd_rocclr_copyBuffer"


def test_bytes_per_launch_from_scaled_counters(tmp_path):
    kib = 1024
    # copy kernel: 4 GiB moved each way, counters read 2 GiB fetched and 4 GiB written
    _write(tmp_path / "cfetch" / "copy_counter_collection.csv", [(COPY, "FETCH_SIZE", 2 * 1024 * 1024)] * 3)
    _write(tmp_path / "cwrite" / "copy_counter_collection.csv", [(COPY, "WRITE_SIZE", 4 * 1024 * 1024)] * 3)
    L = 2 ** 17
    alg = 3 * L * L * 4 / 8 / 2                              # bytes per launch, 4-bit cells
    read_kib = (2 * L * L * 4 / 8 / 2) * 1.06 / kib / 2.0    # counter value that scales to 1.06x the reads
    write_kib = (L * L * 4 / 8 / 2) * 1.01 / kib
    _write(tmp_path / "fetch" / "bench_counter_collection.csv",
           [(ISING % 0, "FETCH_SIZE", read_kib * 0.99), (ISING % 1, "FETCH_SIZE", read_kib * 1.01)])
    _write(tmp_path / "write" / "bench_counter_collection.csv",
           [(ISING % 0, "WRITE_SIZE", write_kib), (ISING % 1, "WRITE_SIZE", write_kib)])
    out = pmc_summary.main(str(tmp_path))
    assert out["fetch_scale"] == pytest.approx(2.0) and out["write_scale"] == pytest.approx(1.0)
    k = out["sweep_kernels"]["ising_4bit"]
    assert sorted(k["kernels"]) == ["half_sweep_kernel<0, true, 0>", "half_sweep_kernel<0, true, 1>"]
    assert k["algorithmic_bytes_per_launch"] == alg
    assert k["hbm_read_bytes_per_launch"] == pytest.approx(2 * L * L * 4 / 8 / 2 * 1.06)
    assert k["hbm_write_bytes_per_launch"] == pytest.approx(L * L * 4 / 8 / 2 * 1.01)
    assert k["traffic_over_algorithmic"] == pytest.approx((2 * 1.06 + 1.01) / 3)
    assert "blume_capel_4bit" not in out["sweep_kernels"]       # no launches of it in these files
    assert out["kernel_source_sha"] == pmc_summary.source_sha()


def test_valu_figures(tmp_path):
    L = 2 ** 17
    updates = L * L / 2
    cycles = 3.4e-3 * 2.4e9                       # one 3.4 ms launch at 2.4 GHz
    insts = 0.9 * 1024 * cycles / 4               # 90% of the SIMD cycles issuing VALU
    rows = []
    for c in (0, 1):
        rows += [(ISING % c, "SQ_INSTS_VALU", insts), (ISING % c, "SQ_ACTIVE_INST_VALU", insts),
                 (ISING % c, "SQ_INSTS_LDS", 1000.0), (ISING % c, "SQ_LDS_BANK_CONFLICT", 0.25 * 256 * cycles),
                 (ISING % c, "SQ_WAVES", 131072), (ISING % c, "SQ_BUSY_CYCLES", cycles),
                 (ISING % c, "GRBM_GUI_ACTIVE", 8 * cycles)]
    _write(tmp_path / "valu" / "bench_counter_collection.csv", rows)
    v = pmc_summary.valu_summary(str(tmp_path / "valu" / "bench_counter_collection.csv"))["ising_4bit"]
    assert "valu_util" not in v                   # no launch durations given
    durations = {"half_sweep_kernel<0, true, 0>": 3.4e-3, "half_sweep_kernel<0, true, 1>": 3.4e-3}
    v = pmc_summary.valu_summary(str(tmp_path / "valu" / "bench_counter_collection.csv"), durations)["ising_4bit"]
    # 90% of 1024 SIMDs x 2.4 GHz issuing one wave64 instruction per 4 cycles
    assert v["valu_util"] == pytest.approx(0.9)
    assert v["avg_launch_s"] == pytest.approx(3.4e-3)
    assert v["gpu_cycles_per_launch"] == pytest.approx(cycles)
    assert v["valu_lane_ops_per_update"] == pytest.approx(insts * 64 / updates)
    assert v["lds_bank_conflict_share"] == pytest.approx(0.25)


def test_kernel_durations_from_stats(tmp_path):
    path = tmp_path / "bench_kernel_stats.csv"
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Name", "Calls", "TotalDurationNs", "AverageNs"])
        w.writeheader()
        w.writerow({"Name": ISING % 0, "Calls": 2, "TotalDurationNs": 7.0e6, "AverageNs": 3.5e6})
    d = pmc_summary.kernel_durations(str(path))
    assert d == {"half_sweep_kernel<0, true, 0>": pytest.approx(3.5e-3)}
