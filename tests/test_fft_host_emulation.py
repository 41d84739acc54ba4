"""The line FFT engine's own source (paper_1403_3746_amd/csrc/lb_fft.h) built for the CPU: every
supported length, x and y block layouts, one line and several lines at a time, x blocks whose
waves order their exchanges only among themselves, 16 elements per thread (radix-16 passes) for
long lines, 24 elements per thread (a radix-24 pass) for lines of 3*2^a points, 4 elements per
thread (the x pass's alternative plan for lines of 128-512 points),
forward against a naive DFT (the discrete transform the windowed derivative of
Eq. (3) is applied through) and forward-then-inverse against the input.  Runs without a GPU."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "host_fft")
CSRC = os.path.join(ROOT, "paper_1403_3746_amd", "csrc")


@pytest.fixture(scope="module")
def results(tmp_path_factory):
    cxx = shutil.which("g++") or shutil.which("clang++")
    if cxx is None:
        pytest.skip("no host C++ compiler")
    exe = str(tmp_path_factory.mktemp("fftemu") / "fft_emulation")
    cmd = [cxx, "-std=c++20", "-O2", "-I", HERE, "-I", CSRC, os.path.join(HERE, "fft_emulation.cpp"),
           "-o", exe, "-lpthread"]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    out = subprocess.run([exe], check=True, capture_output=True, text=True, timeout=600).stdout
    rows = []
    for line in out.strip().splitlines():
        prec, n, layout, q, ef, er = line.split()
        rows.append((prec, int(n), layout, int(q), float(ef), float(er)))
    return rows


def test_every_case_ran(results):
    sizes = {n for p, n, lay, q, _, _ in results if p == "f64" and lay == "x" and q == 1}
    assert sizes == {8, 12, 16, 24, 32, 48, 64, 96, 128, 192, 256, 384, 512, 768, 1024, 1536, 2048}
    assert len(results) == 2 * 45
    r24 = {(n, lay) for p, n, lay, q, _, _ in results if p == "f32" and lay.endswith("24")}
    assert r24 == {(96, "y24"), (384, "y24"), (192, "xw24"), (384, "xw24")}
    r4 = {(n, lay, q) for p, n, lay, q, _, _ in results if p == "f32" and lay in ("x4", "xw4")}
    assert r4 == {(128, "xw4", 1), (128, "x4", 2), (256, "xw4", 2), (512, "x4", 2)}
    r16 = {(n, lay) for p, n, lay, q, _, _ in results if p == "f32" and lay.endswith("16")}
    assert r16 == {(512, "x16"), (1024, "x16"), (2048, "x16"), (1024, "y16"), (2048, "y16"), (1024, "xw16")}


@pytest.mark.parametrize("prec,tol", [("f64", 4e-15), ("f32", 2.5e-7)])
def test_forward_matches_naive_dft(results, prec, tol):
    import math
    for p, n, lay, q, ef, _ in results:
        if p == prec:
            assert ef < tol * (1 + math.log2(n)), (p, n, lay, q, ef)


@pytest.mark.parametrize("prec,tol", [("f64", 2e-15), ("f32", 1.5e-7)])
def test_round_trip_returns_input(results, prec, tol):
    import math
    for p, n, lay, q, _, er in results:
        if p == prec:
            assert er < tol * (1 + math.log2(n)), (p, n, lay, q, er)
