"""Build of the HIP library libmppi_jump.so for gfx950 (in-tree)."""

import os
import shutil
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(HERE, "csrc", "mppi_jump.hip")
LIB = os.path.join(HERE, "libmppi_jump.so")

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # packed fp32 instructions are kept out of every kernel
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result",
]


def hipcc():
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def build(extra_flags=(), out=LIB, verbose=False):
    """Compile the library; returns its path.  Always recompiles."""
    tmp = out + ".tmp"
    cmd = [hipcc()] + HIPCC_FLAGS + list(extra_flags) + ["-I", os.path.join(ROOT, "include"),
                                                         "-o", tmp, SRC]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


PROBE_SRC = os.path.join(HERE, "probe", "issue_rates.hip")
PROBE_BIN = os.path.join(HERE, "probe", "issue_rates")


def build_probe(verbose=False):
    """Compile the VALU issue-rate probe (an executable for gfx950)."""
    cmd = [hipcc(), "--offload-arch=gfx950", "-O3", "-Xclang", "-target-feature", "-Xclang",
           "-packed-fp32-ops", "-o", PROBE_BIN, PROBE_SRC]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    return PROBE_BIN


if __name__ == "__main__":
    print(build(verbose=True))
    print(build_probe(verbose=True))
