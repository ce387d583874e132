"""Build the HIP library ``libmcl.so`` for gfx950 with hipcc (in-tree)."""
from __future__ import annotations

import os
import shutil
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libmcl.so")
SOURCES = ["api.hip", "sweep.hip", "measure.hip", "batch.hip"]  # calibrate.hip is a separate program

# Packed-FP32 instructions are switched off for all device code; the
# library has no floating point on the device, but the flag keeps the
# compiler from ever emitting them.
HIP_FLAGS = ["-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC", "-Wall",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def hipcc() -> str:
    exe = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(exe):
        raise RuntimeError("hipcc not found; the HIP library cannot be built")
    return exe


def build_library(extra_flags=None, out=LIB, verbose=False) -> str:
    srcs = [os.path.join(CSRC, s) for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]
    tmp = out + ".tmp%d" % os.getpid()
    cmd = [hipcc(), *HIP_FLAGS, *(extra_flags or []), "-shared", "-I", os.path.join(ROOT, "include"),
           "-o", tmp, *srcs]
    if verbose:
        print(" ".join(cmd))
    res = subprocess.run(cmd, cwd=CSRC, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + res.stdout + res.stderr)
    os.replace(tmp, out)
    return out


CALIBRATE = os.path.join(HERE, "mcl_calibrate")


def build_calibrate(out=CALIBRATE) -> str:
    """Standalone calibration program (copy / Philox / VALU rates)."""
    tmp = out + ".tmp%d" % os.getpid()
    cmd = [hipcc(), *HIP_FLAGS, "-o", tmp, os.path.join(CSRC, "calibrate.hip")]
    res = subprocess.run(cmd, cwd=CSRC, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + res.stdout + res.stderr)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build_library(verbose=True))
    print(build_calibrate())
