"""Quench with energy history (Sec. 3.2) on the GPU: the step at the run's own parameters
(dt/tau = 1, dx = 1/256, the rings scaled for T near 1) against the FP64 oracle, and a short run
of `quench.run` whose per-step history is checked against the oracle's integrals."""
import numpy as np
import pytest

from oracle import model
from paper_1403_3746_amd import quench as Q
from tests.gpu_util import say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _params():
    p = dict(Q.PAPER_PARAMS)
    p["dvm"] = Q.QUENCH_DVM
    return p


def test_quench_step_matches_oracle(torch_cuda):
    from paper_1403_3746_amd.lbfft import Sim
    p = _params()
    ic = Q.initial(128, seed=7)
    sim = Sim([(p, ic)], "fp64", dvm=Q.QUENCH_DVM)
    f = model.init_equilibrium(*ic, p)
    for n in range(3):
        sim.step(1)
        f = model.rk2_step(f, p)
        g = sim.get_f()
        err = np.abs(g - f).max() / np.abs(f).max()
        say(f"quench params step {n + 1}: rel err {err:.2e}")
        assert err < 1e-12
    sim.close()


def test_short_quench_history(torch_cuda):
    p = _params()
    r = Q.run(t_end=0.2, chunk=500, every=100, snap_times=(0.05, 0.2), seed=7)
    assert r["steps"] == 2000 and r["failed_at"] is None and len(r["times"]) == 20 and r["times"][:2] == pytest.approx([0.0, 0.01])
    c0 = model.conservation(model.init_equilibrium(*Q.initial(128, seed=7), p), p)
    assert abs(r["e0"] - c0[3]) < 1e-12 * abs(c0[3]), (r["e0"], c0[3])
    assert abs(r["e_T"][0] - c0[3]) < 1e-12 * abs(c0[3])
    say(f"quench t=0.2: max|de_T| {r['max_abs_de']:.3e} of e_T {r['e0']:.6f}; mass drift "
        f"{r['mass_drift']:.1e}; snapshots {r['snapshots']}")
    assert r["mass_drift"] < 1e-13 * abs(c0[0])
    assert r["max_abs_de"] < 1e-8 * abs(c0[3])
    assert set(r["snapshots"]) == {0.05, 0.2} and r["rho"][0.2].shape == (128, 128)
