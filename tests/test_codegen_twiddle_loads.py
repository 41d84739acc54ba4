"""Code-generation guard for the line kernels (no GPU): hipcc of ROCm 7.2 once paired the halves
of two different twiddle-table entries when a complex entry was read as two 8-byte loads (the
96-point float64 x passes then took butterfly 3's imaginary twiddle from butterfly 5's entry; the
optimised IR was right).  Table entries are now read with one load per complex word.  This test
compiles the line-kernel units to gfx950 assembly with the library's flags and checks every
kernel for that fault's signature: an 8-byte load that re-reads part of a 16-byte load (or the
reverse) from the same address operand, with the address register not rewritten in between."""
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
LOAD = re.compile(r"global_load_dwordx(\d) (v\[\d+:\d+\]), (v\[\d+:\d+\]|v\d+), (off|s\[\d+:\d+\])"
                  r"(?: offset:(\d+))?")


def _vregs(op):
    m = re.match(r"v\[(\d+):(\d+)\]", op)
    if m:
        return set(range(int(m.group(1)), int(m.group(2)) + 1))
    m = re.match(r"v(\d+)$", op)
    return {int(m.group(1))} if m else set()


def _assembly(unit, out_dir):
    out = os.path.join(out_dir, unit + ".s")
    cmd = [B.HIPCC] + [f for f in B.FLAGS if f != "-fPIC"] + ["--offload-device-only", "-S",
                                                              os.path.join(B.CSRC, unit + ".hip"), "-o", out]
    subprocess.run(cmd, check=True, capture_output=True, text=True, timeout=600)
    return open(out).read()


def half_reloads(asm):
    """Kernels with an 8-byte global load inside a 16-byte one (either order) from the same
    address operand (vector address or offset register plus scalar base) while that address
    register is not rewritten in between."""
    bad = []
    for m in re.finditer(r"^(_ZN5lbfft\w+):\s*;", asm, re.M):
        end = asm.find("s_endpgm", m.end())
        live = {}   # address operand -> (width, offset) of the loads since its last write
        for line in asm[m.end():end].splitlines():
            line = line.strip()
            if not line or line.startswith((";", ".")):
                continue
            parts = re.split(r"[\s,]+", line)
            ld = LOAD.match(line)
            if ld:
                w, base, sbase, off = int(ld.group(1)), ld.group(3), ld.group(4), int(ld.group(5) or 0)
                for w2, o2 in live.get((base, sbase), []):
                    if (w == 2 and w2 == 4 and o2 <= off and off + 8 <= o2 + 16) or \
                       (w == 4 and w2 == 2 and off <= o2 and o2 + 8 <= off + 16):
                        bad.append(m.group(1))
                live.setdefault((base, sbase), []).append((w, off))
            # a vector instruction or load rewrites its first operand's registers
            if parts[0].startswith(("v_", "global_load", "buffer_load", "ds_read", "scratch_load")) and len(parts) > 1:
                written = _vregs(parts[1])
                for key in [k for k in live if _vregs(k[0]) & written]:
                    del live[key]
    return sorted(set(bad))


def test_signature_detector_finds_a_planted_reload():
    # the pattern the faulty code had, in synthetic kernel bodies: caught with an offset register
    # and with a 64-bit address, in either order; not when the address is recomputed in between
    asm = ("_ZN5lbfft4testEv: ; @x\n  global_load_dwordx4 v[12:15], v16, s[10:11]\n"
           "  global_load_dwordx2 v[144:145], v16, s[10:11] offset:8\n  s_endpgm\n"
           "_ZN5lbfft5test2Ev: ; @x\n  global_load_dwordx2 v[20:21], v[2:3], off offset:8\n"
           "  global_load_dwordx4 v[12:15], v[2:3], off\n  s_endpgm\n"
           "_ZN5lbfft5cleanEv: ; @y\n  global_load_dwordx4 v[12:15], v16, s[10:11]\n"
           "  global_load_dwordx2 v[144:145], v17, s[10:11] offset:8\n  s_endpgm\n"
           "_ZN5lbfft6clean2Ev: ; @y\n  global_load_dwordx4 v[12:15], v[2:3], off\n"
           "  v_lshl_add_u64 v[2:3], v[4:5], 3, v[0:1]\n"
           "  global_load_dwordx2 v[20:21], v[2:3], off offset:8\n  s_endpgm\n")
    assert half_reloads(asm) == ["_ZN5lbfft4testEv", "_ZN5lbfft5test2Ev"]


def test_no_line_kernel_rereads_half_a_complex_load(tmp_path):
    if not os.path.exists(B.HIPCC) and shutil.which("hipcc") is None:
        pytest.skip("hipcc not available")
    with ThreadPoolExecutor(len(UNITS)) as ex:
        asms = list(ex.map(lambda u: _assembly(u, str(tmp_path)), UNITS))
    bad = {u: half_reloads(a) for u, a in zip(UNITS, asms)}
    assert all(len(re.findall(r"^_ZN5lbfft\w+:", a, re.M)) > 10 for a in asms)
    assert not any(bad.values()), bad
