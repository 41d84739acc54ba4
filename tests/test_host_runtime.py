"""CPU check of the host runtime (argument handling, workspace carving, job tables, stage
sequencing, graph capture bookkeeping, timing hooks, history, free) under AddressSanitizer and
UBSan: lb_runtime's source is compiled with g++ against a small host mock of the HIP API
(tests/host_mock) whose copies are memcpy and whose kernel launches are argument-checked no-ops."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
MOCK = os.path.join(ROOT, "tests", "host_mock")
CSRC = os.path.join(ROOT, "paper_1403_3746_amd", "csrc")


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_host_runtime_under_sanitizers(tmp_path):
    # copy the runtime source to a .cpp file: the host compiler builds it as plain C++
    src = tmp_path / "lb_runtime_host.cpp"
    shutil.copy(os.path.join(CSRC, "lb_runtime.hip"), src)
    exe = tmp_path / "runtime_check"
    cmd = ["g++", "-std=c++17", "-g", "-O1", "-fsanitize=address,undefined", "-fno-sanitize-recover",
           "-I", MOCK, "-I", CSRC, "-I", os.path.join(ROOT, "include"),
           str(src), os.path.join(MOCK, "mock_launch.cpp"), os.path.join(MOCK, "driver.cpp"),
           "-o", str(exe)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, (r.stdout + r.stderr)[-4000:]
    lines = r.stdout.split("\n")
    assert "init 0 " in lines and "init2 0 " in lines and "init3 0 0" in lines and "done" in lines, r.stdout
    assert "setmom 0" in lines and "setmom_bad -1" in lines, r.stdout
