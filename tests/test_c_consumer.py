"""The C ABI from a plain C99 program: tests/c_consumer.c is compiled with gcc
against include/csl.h, linked to the in-tree libcsl.so and run (host entry
points only, no GPU)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIBDIR = os.path.join(ROOT, "paper_2408_00488_amd")


def test_c_program_uses_the_abi(tmp_path):
    gcc = shutil.which("gcc")
    if gcc is None or not os.path.exists("/opt/rocm/include/hip/hip_runtime_api.h"):
        pytest.skip("gcc or the HIP headers are not available")
    if not os.path.exists(os.path.join(LIBDIR, "libcsl.so")):
        pytest.skip("libcsl.so is not built")
    exe = tmp_path / "c_consumer"
    cmd = [gcc, "-std=c99", "-O1", "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(ROOT, "include"),
           "-I", "/opt/rocm/include", os.path.join(ROOT, "tests", "c_consumer.c"),
           "-L", LIBDIR, "-lcsl", "-lm", "-Wl,-rpath," + LIBDIR, "-o", str(exe)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=60)
    assert r.returncode == 0 and r.stdout.strip() == "ok", (r.returncode, r.stdout, r.stderr[-2000:])
