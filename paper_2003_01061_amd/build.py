"""Build libsphmesh.so (the gfx950 HIP kernels and the C ABI) in-tree.

hipcc cross-compiles for gfx950 without a GPU.  Packed FP32 instructions are
disabled (-packed-fp32-ops); the FP32 path uses scalar FP32 VALU.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libsphmesh.so")
SOURCES = [os.path.join(HERE, "csrc", "sph_mesh.hip")]
DEPS = SOURCES + [os.path.join(HERE, "csrc", "sph_device.h"), os.path.join(HERE, "csrc", "sph_kernels.h"),
                  os.path.join(HERE, "csrc", "sph_setup.h"),
                  os.path.join(HERE, "csrc", "sph_tags.h"),
                  os.path.join(ROOT, "include", "sph_mesh.h")]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = os.environ.get("SPH_OFFLOAD_ARCH", "gfx950")


def flags():
    return ["--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC", "-shared",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-munsafe-fp-atomics", "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
            "-Wno-unused-result", "-Wshadow",
            "-I" + os.path.join(ROOT, "include")]


def stale():
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    return any(os.path.getmtime(p) > t for p in DEPS)


def build(force=True, verbose=False):
    if not force and not stale():
        return LIB
    cmd = [HIPCC] + flags() + SOURCES + ["-o", LIB + ".tmp"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
