"""Build of the HIP library libmppi_jump.so for gfx950 (in-tree), of its
phase-profiling variant and of the issue-rate probe."""

import os
import shutil
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(HERE, "csrc", "mppi_jump.hip")
LIB = os.path.join(HERE, "libmppi_jump.so")

# Packed fp32 instructions are kept out of every kernel: a code-generation
# feature of the gfx950 device pass.  hipcc cannot forward "-Xclang" options
# to one pass only (-Xarch_device refuses options that take an argument), so
# the host (x86) pass sees the feature too, ignores it and says so; run()
# drops that one notice from the build log.
NO_PACKED_FP32 = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
HOST_PASS_NOTICE = "'-packed-fp32-ops' is not a recognized feature for this target"

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    *NO_PACKED_FP32,
    "-Wall", "-Wno-unused-result",
]


def run(cmd, verbose=False):
    """Run one compiler command; its diagnostics are printed except the host
    pass's notice about the device-only feature.  Raises on failure."""
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    out = [ln for ln in r.stdout.splitlines() if HOST_PASS_NOTICE not in ln]
    if out:
        print("\n".join(out), flush=True)
    if r.returncode != 0:
        raise subprocess.CalledProcessError(r.returncode, cmd)


def hipcc():
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


# The phase-profiling build: the same sources with per-workgroup phase
# timestamps compiled in (MPPI_PHASE_STAMPS; include/mppi_jump_phases.h),
# loaded only by phase_profile.py.
PHASE_LIB = os.path.join(HERE, "libmppi_jump_phases.so")


def build(extra_flags=(), out=LIB, verbose=False):
    """Compile the library; returns its path.  Always recompiles."""
    tmp = out + ".tmp"
    cmd = [hipcc()] + HIPCC_FLAGS + list(extra_flags) + ["-I", os.path.join(ROOT, "include"),
                                                         "-o", tmp, SRC]
    run(cmd, verbose)
    os.replace(tmp, out)
    return out


def build_phases(verbose=False):
    """Compile the phase-profiling library; returns its path."""
    return build(extra_flags=["-DMPPI_PHASE_STAMPS"], out=PHASE_LIB, verbose=verbose)


# Measurement probe (an executable for gfx950): the VALU issue rates of the
# instruction classes the rollout uses, the calibration of its roofline peak.
PROBES = ("issue_rates",)


def build_probe(verbose=False):
    """Compile the measurement probe; returns its path(s)."""
    out = []
    for name in PROBES:
        src = os.path.join(HERE, "probe", name + ".hip")
        bin_ = os.path.join(HERE, "probe", name)
        run([hipcc(), "--offload-arch=gfx950", "-O3", *NO_PACKED_FP32, "-o", bin_, src], verbose)
        out.append(bin_)
    return out


if __name__ == "__main__":
    print(build(verbose=True))
    print(build_phases(verbose=True))
    print(build_probe(verbose=True))
