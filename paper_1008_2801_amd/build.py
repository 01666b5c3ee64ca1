"""Build the gfx950 shared libraries libppm.so (the step) and libppm_diag.so
(its arithmetic diagnostics) in-tree with hipcc.

Flags: -O3, no FP contraction (the step's formulas are evaluated exactly as
written), no packed FP32 instructions, position-independent shared object.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = [os.path.join(HERE, "csrc", f) for f in ("ppm_api.hip", "ppm_kernels.hip", "ppm_adjoint.hip", "ppm_species.hip", "ppm_amr.hip")]
OUT = os.path.join(HERE, "libppm.so")
# the arithmetic diagnostics (include/ppm_diag.h), a library of their own
DIAG_SRC = [os.path.join(HERE, "csrc", "ppm_diag.hip")]
DIAG_OUT = os.path.join(HERE, "libppm_diag.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

FLAGS = ["-O3", "-std=c++17", "-fPIC", "-shared", f"--offload-arch={ARCH}", "-ffp-contract=off",
         "-fno-fast-math", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I", os.path.join(ROOT, "include"), "-I", os.path.join(HERE, "csrc"), "-Wall"]


def build(verbose=False):
    for src, out in ((SRC, OUT), (DIAG_SRC, DIAG_OUT)):
        cmd = [HIPCC] + FLAGS + src + ["-o", out + ".tmp"]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd)
        os.replace(out + ".tmp", out)
    return OUT


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
