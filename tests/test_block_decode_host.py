"""The line passes' block decoding (paper_1403_3746_amd/csrc/lb_decode.h) built for the CPU: each
(instance, tile, job) of a launch is taken by exactly one block, on the XCD that owns its group, in
both block orders.  Runs without a GPU."""
import os
import shutil
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "host_fft")
CSRC = os.path.join(ROOT, "paper_1403_3746_amd", "csrc")


def test_block_decoding_covers_every_job_once(tmp_path):
    cxx = shutil.which("g++") or shutil.which("clang++")
    assert cxx is not None, "no host C++ compiler"
    exe = str(tmp_path / "decode_check")
    subprocess.run([cxx, "-std=c++20", "-O2", "-I", HERE, "-I", CSRC,
                    os.path.join(HERE, "decode_check.cpp"), "-o", exe], check=True,
                   capture_output=True, text=True)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    lines = r.stdout.split()
    assert "group_major" in lines and "job_major" in lines, r.stdout
