"""Coexistence-curve driver (Sec. 3.1) on the GPU: the restart-from-moments entry point against
the oracle's equilibrium, and a short run of the quasi-1-D slab near the van der Waals
coexistence densities of the paper's fluid (Maxwell construction from the oracle's EOS)."""
import numpy as np
import pytest

from oracle import dvm as odvm
from oracle import eos, model
from paper_1403_3746_amd import coexistence as cx
from paper_1403_3746_amd import workloads as W
from tests.gpu_util import say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-13), ("fp32", 2e-6)])
def test_set_moments_is_the_equilibrium_of_the_fields(torch_cuda, prec, tol):
    from paper_1403_3746_amd.lbfft import LBError, Sim
    p = W.base_params()
    sim = Sim([(p, W.quench(48, 32, 0.5, 3))], prec)
    sim.step(3)
    rho, ux, uy, T = W.smooth_random(48, 32, 11, T0=0.52)
    sim.set_moments(rho, ux, uy, T)
    f = sim.get_f()
    ref = model.init_equilibrium(rho, ux, uy, T, p)
    err = np.abs(f - ref).max() / np.abs(ref).max()
    say(f"set_moments {prec}: f vs oracle f^eq rel err {err:.2e}")
    assert err < tol
    # the moments of the new state are the given fields
    r2, x2, y2, T2 = sim.moments()
    assert np.abs(r2 - rho).max() / rho.max() < 10 * tol and np.abs(T2 - T).max() / T.max() < 10 * tol
    # invalid fields are refused and leave the state as it was
    bad = T.copy()
    bad[5, 7] = -1.0
    with pytest.raises(LBError):
        sim.set_moments(rho, ux, uy, bad)
    assert np.array_equal(sim.get_f(), f)
    sim.close()


def test_fp32_temperature_far_from_its_reference(torch_cuda):
    # an FP32 context stores T as its deviation from the reference temperature of its initial
    # state (0.5 here).  Restarted at T ~ 0.9 (deviation 0.4) it reads the moments back to float32
    # rounding, and the parts that add the reference back match an FP64 context on the same state:
    # B, C + C_q (stress and finalize kernels), R(f) (the x pass's equilibrium), the conservation
    # sums.  tau = 1 keeps the rounding of R's BGK term unamplified (the oracle puts the effect of
    # float32 moments at 2e-6 of max|R|; with T off by 0.4 R would move by 11 max|R|, B by 4 max|B|
    # and C by 0.8 max|C|).
    from paper_1403_3746_amd.lbfft import Sim
    p = W.base_params(q=-0.004, H=1e-3, tau=1.0)
    ic = W.quench(48, 32, 0.5, 3)
    rho, ux, uy, T = W.smooth_random(48, 32, 12, T0=0.9)
    out = {}
    for prec in ("fp32", "fp64"):
        sim = Sim([(p, ic)], prec)
        sim.step(2)
        sim.set_moments(rho, ux, uy, T)
        out[prec] = (sim.moments(), sim.force_coefficients(), sim.rhs(), sim.conservation())
        sim.close()
    (r2, x2, y2, T2), F32, R32, c32 = out["fp32"]
    _, F64, R64, c64 = out["fp64"]
    eT = np.abs(T2 - T).max() / T.max()
    eF = [np.abs(a - b).max() / np.abs(b).max() for a, b in zip(F32, F64)]
    eR = np.abs(R32 - R64).max() / np.abs(R64).max()
    eE = abs(c32[3] - c64[3]) / abs(c64[3])
    say(f"fp32 at T - T_ref ~ 0.4: T readback {eT:.2e}, B_x B_y C vs fp64 {eF}, R(f) {eR:.2e}, "
        f"energy {eE:.2e}")
    assert np.abs(r2 - rho).max() / rho.max() < 2e-6 and eT < 2e-6
    assert eF[0] < 5e-4 and eF[1] < 5e-4 and eF[2] < 1e-3   # measured 8e-5, 6e-5, 5e-6
    assert eR < 1e-4   # measured 1.5e-5
    assert abs(c32[0] - c64[0]) < 1e-6 * abs(c64[0]) and eE < 1e-5


def test_slab_near_maxwell_coexistence(torch_cuda):
    # a liquid slab at the Maxwell densities of T = 0.9, with the interface resolved (K = 1e-4 on
    # the Sec. 3.1 grid); after the run the bulk densities stay near the Maxwell values
    T = 0.9
    rv, rl = eos.maxwell(T, 9 / 8, 1 / 3)
    x = np.arange(512)
    prof = 0.5 * (rl + rv) + 0.5 * (rl - rv) * np.tanh((128 - np.abs(x - 256.5)) / 2.0)
    rho = np.vstack([prof, prof])
    z = np.zeros_like(rho)
    rec, = cx.run([T], params=dict(K=1e-4), ic=(rho, z, z, np.full_like(rho, T)), check=5000,
                  window=4, max_steps=150000)
    say(f"coexistence T=0.9 K=1e-4: rho_v {rec['rho_v']:.5f} (Maxwell {rv:.5f}) "
        f"rho_l {rec['rho_l']:.5f} (Maxwell {rl:.5f}) after {rec['steps']} steps")
    assert abs(rec["rho_l"] / rl - 1) < 0.003
    assert abs(rec["rho_v"] / rv - 1) < 0.01
