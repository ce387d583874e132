"""Host logic of bench.py (CPU only): the one-GPU guard, the batched
replica set, the PMC record and its kernel-source check, and the parsing of
the calibration program's output."""
import json
import os
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in (r.stdout + r.stderr)


def test_replica_set_is_the_stated_workload():
    reps = bench.replica_set()
    assert len(reps) == 512
    assert [m for m, *_ in reps] == [i % 2 for i in range(512)]             # alternating Ising / Blume-Capel
    assert {L for _, L, *_ in reps} == {512, 1024, 2048, 4096, 8192}
    assert [s for _, _, s, _, _ in reps] == [2000 + i for i in range(512)]
    for m, L, s, beta, D in reps:
        T = 1.0 / beta
        assert 0.5 / bench.BETA_C <= T <= 1.5 / bench.BETA_C
        assert D in ((0.0,) if m == 0 else (0.0, 0.5, 1.0))
    assert reps == bench.replica_set()                                       # seeded


def _fake_tree(tmp_path, sha_matches):
    for f in bench.SWEEP_SOURCES:
        p = tmp_path / f
        p.parent.mkdir(parents=True, exist_ok=True)
        p.write_text("// %s\n" % f)
    (tmp_path / "profiles").mkdir()
    rec = {"kernel_source_sha": "0" * 16,
           "sweep_kernels": {"ising_4bit": {"hbm_bytes_per_launch": 13.55e9, "valu_util": 0.9978}}}
    if sha_matches:
        old = bench.ROOT
        bench.ROOT = str(tmp_path)
        try:
            rec["kernel_source_sha"] = bench.kernel_source_sha()
        finally:
            bench.ROOT = old
    (tmp_path / "profiles" / "traffic_sweep_kernels.json").write_text(json.dumps(rec))


@pytest.mark.parametrize("current", [True, False])
def test_pmc_record_only_for_the_kernel_source_it_was_taken_on(tmp_path, monkeypatch, current):
    _fake_tree(tmp_path, current)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    if current:
        assert bench.measured_traffic("ising_4bit") == 13550000000
        assert bench.measured_valu_util("ising_4bit") == 0.998
        assert bench.traffic_source().endswith("current")
    else:
        assert bench.measured_traffic("ising_4bit") is None
        assert bench.measured_valu_util("ising_4bit") is None
        assert "stale" in bench.traffic_source()
    assert bench.measured_traffic("no_such_kernel") is None


def test_missing_pmc_summary(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.measured_traffic("ising_4bit") is None
    assert bench.traffic_source().startswith("no PMC summary")


def test_calibration_output_is_parsed(monkeypatch):
    outputs = {
        "copy": "device gfx950\ncopy 4GiB->4GiB: 1.830 ms  4694.5 GB/s\ncopy 4GiB->4GiB: 1.791 ms  4796.0 GB/s\n",
        "philox": "philox variant 0 (library: mad_u64 + bitop3): 1.2 ms  866.9 Gblocks/s = 3467.7 draws/ns\n"
                  "philox attainable: 884.6 Gblocks/s\n",
    }
    monkeypatch.setattr(bench, "_calibrate", lambda mode: outputs[mode])
    assert bench.attainable_copy() == 4796.0
    assert bench.attainable_philox() == 884.6
    monkeypatch.setattr(bench, "_calibrate", lambda mode: "")
    assert bench.attainable_copy() is None and bench.attainable_philox() is None
