"""Host logic of the plan builder, on the CPU: the contraction work lists.

tests/host/work_lists.cpp includes the plan builder's source and checks, for
band-limits 1..260 and a set of larger ones and spins, that every segment of
every chain group is listed exactly once, in a consistent slot layout, with
restart boundaries on checkpoint planes, and that lists which fit the GPU at
once spread their steps over the compute units."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")


def test_work_lists(tmp_path):
    gxx = shutil.which("g++")
    if gxx is None or not os.path.isdir(os.path.join(ROCM, "include", "hip")):
        pytest.skip("needs g++ and the HIP headers")
    exe = str(tmp_path / "work_lists")
    subprocess.check_call([gxx, "-O2", "-std=c++17", "-I", os.path.join(ROOT, "include"),
                           "-I", os.path.join(ROCM, "include"), "-D__HIP_PLATFORM_AMD__",
                           os.path.join(ROOT, "tests", "host", "work_lists.cpp"), "-o", exe,
                           "-L", os.path.join(ROCM, "lib"), "-lamdhip64"])
    env = dict(os.environ)
    env["LD_LIBRARY_PATH"] = os.path.join(ROCM, "lib") + ":" + env.get("LD_LIBRARY_PATH", "")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-2000:]
    assert r.stdout.strip().endswith(" 0 problems"), r.stdout[-3000:]
