"""Build the CPU oracle (test infrastructure) as oracle/libsphref.so.

gcc, -O2, no FMA contraction (-ffp-contract=off) and no fast-math, so every
expression in sphref.c rounds exactly as written.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "libsphref.so")


def build(force=True, sanitize=False):
    src = os.path.join(HERE, "sphref.c")
    if not force and os.path.exists(LIB) and os.path.getmtime(LIB) >= os.path.getmtime(src):
        return LIB
    cmd = ["gcc", "-std=c11", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
           "-Wall", "-Wextra", "-Wno-unused-parameter", "-D_GNU_SOURCE", src, "-o", LIB + ".tmp", "-lm"]
    if sanitize:
        cmd[1:1] = ["-fsanitize=address,undefined", "-fno-omit-frame-pointer", "-g"]
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(sanitize="--sanitize" in sys.argv))
