"""Build the CPU oracle library (test infrastructure only).

Plain gcc, FP64, no fast-math and no floating-point contraction, OpenMP over
independent targets.  Produces ``oracle/liboracle.so``.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SOURCES = ["fmm_oracle.c", "mlp_oracle.c"]
LIB = os.path.join(HERE, "liboracle.so")


def build(verbose=False, sanitize=False, out=None):
    """sanitize: AddressSanitizer and UndefinedBehaviorSanitizer instrumentation
    (for the CPU test that runs the oracle under them; the Python process then
    needs libasan preloaded).  out: the library path (default oracle/liboracle.so)."""
    lib = out or LIB
    srcs = [os.path.join(HERE, s) for s in SOURCES]
    cmd = ["gcc", "-std=gnu11", "-O2", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
           "-fcx-fortran-rules", "-fno-fast-math", "-Wall"]
    if sanitize:
        cmd += ["-fsanitize=address,undefined", "-fno-omit-frame-pointer",
                "-fno-sanitize-recover=undefined"]
    cmd += ["-o", lib + ".tmp"] + srcs + ["-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(lib + ".tmp", lib)
    return lib


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
