"""The plan code of the C ABI (validation, static orders, bit packing of 32-,
64- and 128-bit rows, root classes, workspace layout) under AddressSanitizer
and UndefinedBehaviorSanitizer, on the CPU.  tests/host_asan/plan_driver.cpp
stubs the kernels out and drives mcs_plan_create / mcs_plan_root_bounds /
mcs_workspace_size over graphs of 0..128 vertices, directed or not, with 0, 3
or 70 labels, in both static orders, plus rejected inputs."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
ROCM = "/opt/rocm"


def test_plan_code_is_clean_under_sanitizers(tmp_path):
    gxx = shutil.which("g++")
    if gxx is None or not os.path.exists(os.path.join(ROCM, "lib", "libamdhip64.so")):
        pytest.skip("needs g++ and the HIP runtime library")
    exe = str(tmp_path / "plan_driver")
    cmd = [gxx, "-std=c++17", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=undefined", "-g", "-O1", "-D__HIP_PLATFORM_AMD__",
           "-I", os.path.join(ROCM, "include"), "-I", os.path.join(ROOT, "include"),
           "-I", os.path.join(ROOT, "paper_1908_06418_amd", "csrc"),
           os.path.join(HERE, "host_asan", "plan_driver.cpp"),
           os.path.join(ROOT, "paper_1908_06418_amd", "csrc", "mcs_host.cpp"),
           "-L", os.path.join(ROCM, "lib"), "-lamdhip64",
           "-Wl,-rpath," + os.path.join(ROCM, "lib"), "-o", exe]
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    assert r.returncode == 0, r.stdout[-4000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0", HIP_VISIBLE_DEVICES="")
    r = subprocess.run([exe], stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True,
                       env=env, timeout=600)
    assert r.returncode == 0 and "host plan checks passed" in r.stdout, r.stdout[-4000:]
