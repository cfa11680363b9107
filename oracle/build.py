"""Compile the CPU oracle (plain C) into oracle/liboracle.so.

TEST INFRASTRUCTURE ONLY: the oracle is the independent CPU reference used by
the tests, the smoke check and the CPU-baseline leg of the benchmark.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = ["evo_stats.c", "evo_scene.c", "evo_bvh.c", "evo_render.c", "evo_batch.c", "evo_diff.c"]
LIB = os.path.join(HERE, "liboracle.so")


def build(verbose: bool = False) -> str:
    """Build liboracle.so with gcc; strict IEEE FP32/FP64 (no contraction)."""
    srcs = [os.path.join(HERE, "src", s) for s in SRC]
    tmp = LIB + ".tmp"
    cmd = ["gcc", "-std=gnu11", "-O2", "-fPIC", "-shared", "-pthread",
           "-ffp-contract=off", "-fno-fast-math", "-Wall", "-Wextra",
           "-Wno-unused-parameter", "-o", tmp] + srcs + ["-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
