"""Build libbp.so (the HIP library) in-tree with hipcc for gfx950."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libbp.so")
SOURCES = ["bp_engine.hip"]
HEADERS = ["bp_kernels.h", "bp_sum.h", "bp_carry.h", "bp_server.h", "bp_tune.h", "bp_lv.h", "bp_lv_run.h",
           "bp_scores.h", "bp_scores_run.h", "bp_repair.h", "bp_repair_run.h", "bp_round.h",
           "bp_round_run.h"]

# -ffp-contract=off: the candidate and sum formulas are evaluated operation
# by operation (no fused multiply-add), as the parity with the CPU reference
# requires.  Packed FP32 instructions are disabled for the whole library.
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-ffp-contract=off", "-fno-fast-math",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I" + os.path.join(ROOT, "include"),
    # roctx ranges around the entry points
    "-L/opt/rocm/lib", "-lrocprofiler-sdk-roctx", "-Wl,-rpath,/opt/rocm/lib",
]


def build(verbose: bool = False) -> str:
    """Compile every source into libbp.so (always recompiles)."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [hipcc] + FLAGS + ["-o", tmp] + [os.path.join(CSRC, s) for s in SOURCES]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    print(LIB)
    sys.exit(0)
