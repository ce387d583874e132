"""Build of the C program tests/c_abi_quench.c: strict C99 with gcc, against
include/mcl.h, libmcl.so and the HIP runtime -- no Python or PyTorch in
the loop.  Used by __graft_entry__.build() and, if the binary is missing,
by the test that runs it."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(HERE, "c_abi_quench.c")
BIN = os.path.join(HERE, "c_abi_quench")
PKG = os.path.join(ROOT, "paper_2502_18624_amd")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")


def build(out=BIN) -> str:
    cmd = ["gcc", "-std=c99", "-O2", "-Wall", "-Wextra", "-Werror", "-D__HIP_PLATFORM_AMD__",
           "-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROCM, "include"), SRC, "-o", out,
           "-L", PKG, "-lmcl", "-L", os.path.join(ROCM, "lib"), "-lamdhip64",
           "-Wl,-rpath," + PKG, "-Wl,-rpath," + os.path.join(ROCM, "lib")]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    return out
