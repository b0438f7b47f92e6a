"""Build the HIP library ``libmhd.so`` for gfx950 with hipcc.

The library is built in-tree (next to this file) so that it travels with
the source tree.  Packed-FP32 instructions are disabled for every HIP
translation unit.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libmhd.so")
SOURCES = ["mhd_lib.hip"]
ARCH = "gfx950"

HIPCC_FLAGS = [
    "--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC", "-shared",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def sources():
    return [os.path.join(CSRC, s) for s in SOURCES]


def build(extra_flags=()) -> str:
    """Compile libmhd.so (always recompiles); returns its path."""
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = ["hipcc", *HIPCC_FLAGS, *extra_flags, "-o", tmp, *sources()]
    subprocess.run(cmd, check=True, cwd=CSRC)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build())
