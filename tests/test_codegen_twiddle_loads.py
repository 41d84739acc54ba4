"""Code-generation guard for the line kernels (no GPU): hipcc of ROCm 7.2 once paired the halves
of two different twiddle-table entries when a complex entry was read as two 8-byte loads (the
96-point float64 x passes then took butterfly 3's imaginary twiddle from butterfly 5's entry; the
optimised IR was right).  Table entries are now read with one load per complex word.  This test
compiles the line-kernel units to gfx950 assembly with the library's flags and checks every
kernel for that fault's signature: an 8-byte load that re-reads part of a 16-byte load from the
same 32-bit offset register and scalar base."""
import os
import re
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
from paper_1403_3746_amd import build as B  # noqa: E402

UNITS = ["lb_lines_x_f64", "lb_lines_x_f32", "lb_lines_y_f64", "lb_lines_y_f32", "lb_lines_xy_f64", "lb_lines_xy_f32"]
LOAD = re.compile(r"global_load_dwordx(\d) (v\[\d+:\d+\]), (v\d+), (s\[\d+:\d+\])(?: offset:(\d+))?")


def _assembly(unit, out_dir):
    out = os.path.join(out_dir, unit + ".s")
    cmd = [B.HIPCC] + [f for f in B.FLAGS if f != "-fPIC"] + ["--offload-device-only", "-S",
                                                              os.path.join(B.CSRC, unit + ".hip"), "-o", out]
    subprocess.run(cmd, check=True, capture_output=True, text=True, timeout=600)
    return open(out).read()


def half_reloads(asm):
    """Kernels with an 8-byte load inside a 16-byte load of the same (offset register, base)."""
    bad = []
    for m in re.finditer(r"^(_ZN5lbfft\w+):\s*;", asm, re.M):
        end = asm.find("s_endpgm", m.end())
        by_base = {}
        for w, _, voff, sbase, off in LOAD.findall(asm[m.end():end]):
            by_base.setdefault((voff, sbase), []).append((int(w), int(off or 0)))
        for loads in by_base.values():
            if any(w == 2 and any(w2 == 4 and o2 <= o and o + 8 <= o2 + 16 for w2, o2 in loads)
                   for w, o in loads):
                bad.append(m.group(1))
                break
    return bad


def test_signature_detector_finds_a_planted_reload():
    # the pattern the faulty code had, in a synthetic kernel body
    asm = ("_ZN5lbfft4testEv: ; @x\n  global_load_dwordx4 v[12:15], v16, s[10:11]\n"
           "  global_load_dwordx2 v[144:145], v16, s[10:11] offset:8\n  s_endpgm\n"
           "_ZN5lbfft5cleanEv: ; @y\n  global_load_dwordx4 v[12:15], v16, s[10:11]\n"
           "  global_load_dwordx2 v[144:145], v17, s[10:11] offset:8\n  s_endpgm\n")
    assert half_reloads(asm) == ["_ZN5lbfft4testEv"]


def test_no_line_kernel_rereads_half_a_complex_load(tmp_path):
    if not os.path.exists(B.HIPCC) and shutil.which("hipcc") is None:
        pytest.skip("hipcc not available")
    with ThreadPoolExecutor(len(UNITS)) as ex:
        asms = list(ex.map(lambda u: _assembly(u, str(tmp_path)), UNITS))
    bad = {u: half_reloads(a) for u, a in zip(UNITS, asms)}
    assert all(len(re.findall(r"^_ZN5lbfft\w+:", a, re.M)) > 10 for a in asms)
    assert not any(bad.values()), bad
