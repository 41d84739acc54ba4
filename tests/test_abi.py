"""The C-ABI library loads and exports every symbol that include/lbfft.h declares (no GPU
calls), and argument checks that need no device."""
import os
import re

import pytest

from paper_1403_3746_amd import lbfft
from paper_1403_3746_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "lbfft.h")).read()
    return sorted(set(re.findall(r"\b(lb_[a-z_0-9]+)\s*\(", src)))


def test_header_and_binding_agree():
    assert set(_declared()) == set(lbfft.EXPORTS)


def test_library_exports_every_declared_symbol():
    lib = lbfft.load()
    for name in _declared():
        assert hasattr(lib, name), name


def test_workspace_bytes_validates_sizes():
    p = W.base_params()
    ok = lbfft.lb_workspace_bytes([lbfft.make_params(p, 64, 64)], lbfft.LB_FP64)
    assert ok > 64 * 64 * 8 * 48
    f32 = lbfft.lb_workspace_bytes([lbfft.make_params(p, 64, 64)], lbfft.LB_FP32)
    assert f32 < ok
    for nx, ny in ((100, 64), (64, 5), (4096, 64), (0, 64), (64, 3)):
        assert lbfft.lb_workspace_bytes([lbfft.make_params(p, nx, ny)], lbfft.LB_FP64) == 0
    for nx, ny in ((512, 2), (96, 1), (2048, 1536)):
        assert lbfft.lb_workspace_bytes([lbfft.make_params(p, nx, ny)], lbfft.LB_FP32) > 0
    bad = dict(p, tau=0.0)
    assert lbfft.lb_workspace_bytes([lbfft.make_params(bad, 64, 64)], lbfft.LB_FP64) == 0
    assert lbfft.lb_workspace_bytes([lbfft.make_params(dict(p, hist=-1), 64, 64)], lbfft.LB_FP64) == 0
    with_hist = lbfft.lb_workspace_bytes([lbfft.make_params(dict(p, hist=1000), 64, 64)], lbfft.LB_FP64)
    assert with_hist >= ok + 1000 * 4 * 8


def test_init_rejects_bad_arguments_without_gpu():
    p = W.base_params()
    rho, ux, uy, T = W.slab(64, 64, 0.5)
    prm = [lbfft.make_params(p, 64, 64)]
    # null workspace -> LB_E_ARG before any device call
    with pytest.raises(lbfft.LBError) as e:
        lbfft.lb_init(prm, lbfft.make_dvm(), lbfft.LB_FP64, [rho], [ux], [uy], [T], 0, 1 << 30, 0)
    assert e.value.status == lbfft.LB_E_ARG
    # non-physical density (1 - b_w rho <= 0) is rejected on the host
    rho_bad = rho.copy()
    rho_bad[3, 3] = 11.0
    with pytest.raises(lbfft.LBError) as e:
        lbfft.lb_init(prm, lbfft.make_dvm(), lbfft.LB_FP64, [rho_bad], [ux], [uy], [T], 256,
                      1 << 30, 0)
    assert e.value.status == lbfft.LB_E_ARG
    # too small a workspace
    with pytest.raises(lbfft.LBError) as e:
        lbfft.lb_init(prm, lbfft.make_dvm(), lbfft.LB_FP64, [rho], [ux], [uy], [T], 256, 1024, 0)
    assert e.value.status == lbfft.LB_E_SIZE


def test_edge_cases_rejected_on_the_host():
    p = W.base_params()
    rho, ux, uy, T = W.slab(64, 64, 0.5)
    prm = [lbfft.make_params(p, 64, 64)]
    # an empty batch needs no workspace and cannot be initialised
    assert lbfft.lb_workspace_bytes([], lbfft.LB_FP64) == 0
    with pytest.raises(lbfft.LBError) as e:
        lbfft.lb_init([], lbfft.make_dvm(), lbfft.LB_FP64, [], [], [], [], 256, 1 << 30, 0)
    assert e.value.status == lbfft.LB_E_ARG
    # without eta on ring 1 the moment matrix of the seven kinetic moments is singular
    with pytest.raises(lbfft.LBError) as e:
        lbfft.lb_init(prm, lbfft.make_dvm(dict(eta0=0.0)), lbfft.LB_FP64, [rho], [ux], [uy], [T],
                      256, 1 << 30, 0)
    assert e.value.status == lbfft.LB_E_ARG and "singular" in str(e.value)
    # 2^a 3^b lengths with more than one factor 3 (36 = 4 * 9) are not supported line lengths
    r36, u36, v36, t36 = W.slab(36, 36, 0.5)
    assert lbfft.lb_workspace_bytes([lbfft.make_params(p, 36, 36)], lbfft.LB_FP64) == 0
    with pytest.raises(lbfft.LBError) as e:
        lbfft.lb_init([lbfft.make_params(p, 36, 36)], lbfft.make_dvm(), lbfft.LB_FP64, [r36], [u36],
                      [v36], [t36], 256, 1 << 30, 0)
    assert e.value.status == lbfft.LB_E_SIZE and "unsupported grid" in str(e.value)
    # calls on a null context fail cleanly
    with pytest.raises(lbfft.LBError) as e:
        lbfft.lb_set_moments(None, 0, rho, ux, uy, T)
    assert e.value.status == lbfft.LB_E_ARG
