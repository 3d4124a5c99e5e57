"""Build libars.so (the HIP library behind include/ars.h) for gfx950.

hipcc cross-compiles without a GPU.  Flags:
  -ffp-contract=on       a * b + c within one source expression becomes one
                         fused multiply-add; contraction never crosses
                         statements, so the kernels that share an expression
                         (fused, reference, batched) still agree bit for bit;
  -packed-fp32-ops off   no packed-FP32 instructions are generated;
  --offload-arch=gfx950  MI355X only.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libars.so")
SOURCES = ["ars_api.hip", "ars_fused.hip", "ars_ref.hip", "ars_reduce.hip", "ars_adjoint.hip", "ars_revolve.hip",
           "ars_batch.hip", "ars_tune.hip", "ars_spectrum.hip", "ars_noalloc.hip",
           "ars_imex.hip", "ars_adjf.hip"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-ffp-contract=on", "-fno-fast-math",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-munsafe-fp-atomics",
    "-Wno-unused-variable", "-Wno-unused-parameter",
]


def sources():
    return [os.path.join(CSRC, s) for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]


def build(verbose: bool = False, extra=()) -> str:
    cmd = [HIPCC] + FLAGS + list(extra) + sources() + ["-o", LIB + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True, extra=sys.argv[1:])
