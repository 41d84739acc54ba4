"""Rectangular droplet (Sec. 3.3) on the GPU, half scale (59 x 7 cells in a 96 x 96 box, the
paper's physical parameters): over the first two time units the droplet contracts along its
long axis, keeps its liquid area, and its temperature stays fixed to a few 1e-3 by the run's
heat conduction."""
import numpy as np
import pytest

from paper_1403_3746_amd import droplet as Dr
from tests.gpu_util import say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def test_half_scale_droplet_contracts(torch_cuda):
    r = Dr.run(t_end=2.0, n=96, length=59, height=7, check_every=2500)
    say(f"droplet aspect {np.round(r['aspect'], 3).tolist()} area {np.round(r['area'], 1).tolist()} "
        f"u_max {r['u_max'][-1]:.2e}")
    assert r["failed_at"] is None and r["steps"] == 20000
    a = np.array(r["aspect"])
    assert a[0] > 7.5 and np.all(np.diff(a) < 0) and a[-1] < 5.0
    area = np.array(r["area"])
    assert np.abs(area / area[0] - 1).max() < 0.02
    assert max(r["T_range"]) < 1e-2
