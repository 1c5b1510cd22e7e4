"""Build the CPU oracle (test infrastructure) as oracle/libsphref.so.

gcc, -O2, no FMA contraction (-ffp-contract=off) and no fast-math, so every
expression in sphref.c rounds exactly as written.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "libsphref.so")
# the same source with its per-particle loops run by OpenMP threads; every
# particle's arithmetic and every reduction's order are those of LIB, so the
# two give bit-identical results (timed as the all-cores CPU baseline)
LIB_OMP = os.path.join(HERE, "libsphref_omp.so")


def build(force=True, sanitize=False, openmp=False):
    src = os.path.join(HERE, "sphref.c")
    out = LIB_OMP if openmp else LIB
    if not force and os.path.exists(out) and os.path.getmtime(out) >= os.path.getmtime(src):
        return out
    cmd = ["gcc", "-std=c11", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
           "-Wall", "-Wextra", "-Wno-unused-parameter", "-D_GNU_SOURCE",
           "-fopenmp" if openmp else "-Wno-unknown-pragmas", src, "-o", out + ".tmp", "-lm"]
    if sanitize:
        cmd[1:1] = ["-fsanitize=address,undefined", "-fno-omit-frame-pointer", "-g"]
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


if __name__ == "__main__":
    print(build(sanitize="--sanitize" in sys.argv))
    print(build(openmp=True))
