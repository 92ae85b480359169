"""Build the HIP library (librrq.so) in-tree for gfx950 with hipcc, and its profiling variant
librrq_phases.so (the same sources with the tile kernel's phase timers, -DRRQ_PHASE_TIMERS)."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "librrq.so")
LIB_PHASES = os.path.join(HERE, "librrq_phases.so")
SOURCES = ["rrq_consts.cpp", "rrq_fit.hip", "rrq_pair.hip", "rrq_batch.hip", "rrq_mlp.hip",
           "rrq_api.hip"]
FLAGS = ["-O3", "--offload-arch=gfx950", "-std=c++17", "-fPIC", "-shared",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def build_library(verbose=False, phase_timers=False):
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    srcs = [os.path.join(CSRC, s) for s in SOURCES]
    lib = LIB_PHASES if phase_timers else LIB
    tmp = lib + ".tmp"
    cmd = [hipcc] + FLAGS + (["-DRRQ_PHASE_TIMERS"] if phase_timers else []) + srcs + ["-o", tmp]
    res = subprocess.run(cmd, cwd=CSRC, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + res.stdout + res.stderr)
    os.replace(tmp, lib)
    if verbose:
        print("built", lib)
    return lib


if __name__ == "__main__":
    build_library(verbose=True)
    build_library(verbose=True, phase_timers=True)
