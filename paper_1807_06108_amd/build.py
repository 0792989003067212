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


# Measurement probes (executables for gfx950): VALU issue rates, dependent
# latencies, and the SIMD placement of a workgroup's wavefronts.
PROBES = ("issue_rates", "dep_latency", "wave_placement")


def build_probe(verbose=False):
    """Compile the measurement probes; returns their paths."""
    out = []
    for name in PROBES:
        src = os.path.join(HERE, "probe", name + ".hip")
        bin_ = os.path.join(HERE, "probe", name)
        cmd = [hipcc(), "--offload-arch=gfx950", "-O3", "-Xclang", "-target-feature", "-Xclang",
               "-packed-fp32-ops", "-o", bin_, src]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        out.append(bin_)
    return out


if __name__ == "__main__":
    print(build(verbose=True))
    print(build_probe(verbose=True))
