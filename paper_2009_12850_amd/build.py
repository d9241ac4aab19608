"""Build libmoncadv.so (all HIP sources, gfx950) in-tree with hipcc."""
from __future__ import annotations

import concurrent.futures as cf
import glob
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libmoncadv.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

# Packed FP32 instructions are disabled for every HIP translation unit.
# Multiply-adds are fused only within one source expression (-ffp-contract=on),
# so a formula gives the same bits wherever the compiler inlines it (the march
# is unrolled by two; with fusion across statements the two copies rounded
# differently and the result depended on the parity of the plane).
# The machine scheduler favours instruction-level parallelism over register
# pressure: the march kernels are bound by issue and latency at two to four
# waves per SIMD, and this ordering measured 2-7 % faster on every form with no
# spills (the register ceilings come from the launch bounds).  The FP64-state
# march instantiations (the step, FP64 source terms, the mixed step, the
# ensemble) are scheduled to group their memory instructions instead, which
# also lowers their register counts: 2-4 % faster on those forms, measured on
# one box against the ILP ordering; the FP32/BF16 march, the work-scaled sweep
# and the learned kernels keep the ILP ordering, which was as fast or faster
# for them.  The step's unit also has the scheduler track register pressure
# with the AMDGPU trackers (the budgeted step 1.3-1.7 % faster on two boxes;
# the other units gained nothing from it).
FLAGS = ["--offload-arch=gfx950", "-O3", "-fPIC", "-std=c++17", "-ffp-contract=on",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-mllvm", "-amdgpu-sched-strategy=max-ilp",
         "-Wall", "-Wno-unused-function", "-Wno-unknown-pragmas"]
MEMORY_CLAUSE_SOURCES = {"march_step64.hip", "march_f64.hip", "march_stepmix.hip",
                         "ensemble.hip"}
RP_TRACKER_SOURCES = {"march_step64.hip"}


def flags_for(src: str) -> list:
    """The compile flags of one source file."""
    name = os.path.basename(src)
    flags = list(FLAGS)
    if name in MEMORY_CLAUSE_SOURCES:
        flags = [("-amdgpu-sched-strategy=max-memory-clause"
                  if f == "-amdgpu-sched-strategy=max-ilp" else f) for f in flags]
    if name in RP_TRACKER_SOURCES:
        flags += ["-mllvm", "-amdgpu-use-amdgpu-trackers=1"]
    return flags


# Extra compile flags for build-time tuning, e.g. MONC_HIPCC_FLAGS=-DMONC_MARCH_WAVES64=4
EXTRA = os.environ.get("MONC_HIPCC_FLAGS", "").split()


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    cmd = [HIPCC, *flags_for(src), *EXTRA, "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")))
    with cf.ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(_compile, srcs))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}")
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
