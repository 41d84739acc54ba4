"""The no-allocation entry point (lb_derivative_noalloc, static device scratch) against the
context entry point it varies (lb_derivative), through the C ABI: two calls in a row, the second
on a smaller grid, both precisions; and its size limit."""
import numpy as np
import pytest

from oracle import spectral
from paper_1403_3746_amd import lbfft
from paper_1403_3746_amd import workloads as W
from tests.gpu_util import rel, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _noalloc(torch, g, dx, prec, axis, order):
    ny, nx = g.shape
    d_g = torch.from_numpy(np.ascontiguousarray(g)).to("cuda")
    d_out = torch.full_like(d_g, float("nan"))
    stream = torch.cuda.current_stream()
    lbfft.lb_derivative_noalloc(nx, ny, dx, prec, axis, order, d_g.data_ptr(), d_out.data_ptr(),
                                stream.cuda_stream)
    torch.cuda.synchronize()
    return d_out.cpu().numpy()


@pytest.mark.parametrize("prec", [lbfft.LB_FP64, lbfft.LB_FP32])
def test_noalloc_derivative_matches_context_entry_point(torch_cuda, prec):
    rng = np.random.default_rng(5)
    dx = 0.37
    name = "fp64" if prec == lbfft.LB_FP64 else "fp32"
    # two calls in a row, the second on a smaller grid; each against lb_derivative of a context of
    # the same grid (the same kernels: bit for bit) and against the oracle
    for (ny, nx, axis, order) in ((256, 384, 0, 1), (64, 32, 1, 2), (512, 2048, 1, 1), (8, 96, 0, 2)):
        g = rng.normal(size=(ny, nx))
        got = _noalloc(torch_cuda, g, dx, prec, axis, order)
        sim = lbfft.Sim([(W.base_params(dx=dx), W.slab(nx, ny, 0.5))], name)
        want = sim.derivative(g, axis, order)
        sim.close()
        ref = spectral.dx_(g, dx) if axis == 0 else spectral.dy_(g, dx)
        if order == 2:
            ref = spectral.dx_(ref, dx) if axis == 0 else spectral.dy_(ref, dx)
        e = rel(got, ref)
        say(f"noalloc {name} {nx}x{ny} axis {axis} order {order}: rel err vs oracle {e:.2e}, "
            f"equal to lb_derivative: {np.array_equal(got, want)}")
        assert np.array_equal(got, want)
        tol = 2e-13 if prec == lbfft.LB_FP64 else 3e-6
        n = nx if axis == 0 else ny
        assert e < tol * (1 + np.log2(n)) / 4


def test_noalloc_derivative_rejects_oversized_and_bad_arguments(torch_cuda):
    d = torch_cuda.zeros(1, dtype=torch_cuda.float64, device="cuda")
    s = torch_cuda.cuda.current_stream().cuda_stream
    with pytest.raises(lbfft.LBError) as e:
        lbfft.lb_derivative_noalloc(2048, 1024, 1.0, lbfft.LB_FP64, 0, 1, d.data_ptr(), d.data_ptr(), s)
    assert e.value.status == lbfft.LB_E_SIZE and "static scratch" in str(e.value)
    with pytest.raises(lbfft.LBError) as e:
        lbfft.lb_derivative_noalloc(100, 64, 1.0, lbfft.LB_FP64, 0, 1, d.data_ptr(), d.data_ptr(), s)
    assert e.value.status == lbfft.LB_E_SIZE
    with pytest.raises(lbfft.LBError) as e:
        lbfft.lb_derivative_noalloc(64, 64, 1.0, lbfft.LB_FP64, 2, 1, d.data_ptr(), d.data_ptr(), s)
    assert e.value.status == lbfft.LB_E_ARG
    with pytest.raises(lbfft.LBError) as e:
        lbfft.lb_derivative_noalloc(64, 64, 1.0, lbfft.LB_FP64, 0, 1, 0, d.data_ptr(), s)
    assert e.value.status == lbfft.LB_E_ARG
