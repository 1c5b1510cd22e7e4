"""The neighbour kernel's hit append (append_hits: hits of a batch of
candidates into a particle's LDS ring column, whole 32-byte list blocks
stored as they complete while the capacity allows) built for the host with
AddressSanitizer and UndefinedBehaviorSanitizer and driven by random hit
patterns for every batch size and ring length the kernels use: the stored
list is the hits in order up to the capacity, no store leaves the list, and
a ring of two blocks or more keeps the last hits the pressure sweep reads.
No GPU."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def test_append_hits_on_the_host(tmp_path):
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    exe = tmp_path / "host_append"
    cmd = [HIPCC, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-I" + os.path.join(ROOT, "include"),
           "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           os.path.join(ROOT, "tests", "host_append.cpp"), "-o", str(exe)]
    subprocess.run(cmd, check=True, capture_output=True)
    res = subprocess.run([str(exe)], capture_output=True, text=True,
                         env=dict(os.environ, ASAN_OPTIONS="detect_leaks=0"))
    assert res.returncode == 0, res.stdout[-2000:] + res.stderr[-4000:]
    assert "runtime error" not in res.stderr, res.stderr[-4000:]
    assert res.stdout.startswith("ok 32000"), res.stdout
