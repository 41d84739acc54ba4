"""Host logic of the quench and droplet drivers without a GPU: initial states, the droplet shape
measure, and the quench driver's chunked reading of the per-step history (sampling, energy and
mass drift, stopping at the first non-finite entry) against a stand-in simulator."""
import numpy as np
import pytest

from paper_1403_3746_amd import droplet as Dr
from paper_1403_3746_amd import quench as Q


def test_quench_initial_state():
    rho, ux, uy, T = Q.initial(128, seed=5)
    assert rho.shape == (128, 128) and np.abs(rho - 1).max() <= 1e-3 and abs(rho.mean() - 1) < 1e-4
    assert np.all(ux == 0) and np.all(uy == 0) and np.all(T == 0.9)
    assert np.array_equal(rho, Q.initial(128, seed=5)[0])


def test_droplet_initial_state_and_shape():
    rho, ux, uy, T = Dr.initial(192)
    assert abs(rho.max() - Dr.RHO_L) < 1e-5 and abs(rho.min() - Dr.RHO_V) < 1e-12
    aspect, area = Dr.shape(rho)
    assert abs(area - 118 * 14) < 10 and 7.5 < aspect < 8.8   # a 118 x 14 box: sqrt(I_x/I_y) = 118/14
    # a disc has aspect 1; an ellipse of semi-axes 30, 15 has 2
    y, x = np.meshgrid(np.arange(128) - 63.5, np.arange(128) - 63.5, indexing="ij")
    disc = np.where(x * x + y * y < 20 ** 2, Dr.RHO_L, Dr.RHO_V)
    ell = np.where((x / 30) ** 2 + (y / 15) ** 2 < 1, Dr.RHO_L, Dr.RHO_V)
    assert abs(Dr.shape(disc)[0] - 1) < 0.01 and abs(Dr.shape(ell)[0] - 2) < 0.02


class FakeQuenchSim:
    """History whose energy drifts linearly and turns NaN at a chosen step."""
    bad_step = None

    def __init__(self, instances, precision, dvm=None):
        (p, _), = instances
        self.hist_len, self.n = p["hist"], 0
        self.ring = []

    def step(self, k):
        for _ in range(k):
            e = -0.05 + 1e-9 * self.n
            row = [1.0, 0.0, 0.0, e]
            if self.bad_step is not None and self.n >= self.bad_step:
                row = [np.nan] * 4
            self.ring.append(row)
            self.n += 1
        self.ring = self.ring[-self.hist_len:]

    def history(self, max_entries, allow_nonfinite=False):
        h = np.array(self.ring[-max_entries:])
        return self.n - len(h), h

    def moments(self):
        return (np.ones((8, 8)),) * 4

    def conservation(self):
        return np.array(self.ring[-1])

    def close(self):
        pass


@pytest.mark.parametrize("bad", [None, 2345])
def test_quench_history_chunks(monkeypatch, bad):
    monkeypatch.setattr(Q.lbfft, "Sim", FakeQuenchSim)
    FakeQuenchSim.bad_step = bad
    r = Q.run(t_end=0.5, chunk=700, every=100, snap_times=(0.1, 0.5), params=dict(dt=1e-4))
    if bad is None:
        assert r["steps"] == 5000 and r["failed_at"] is None
        assert len(r["times"]) == 50 and r["times"][:2] == pytest.approx([0.0, 0.01])
        assert r["max_abs_de"] == pytest.approx(1e-9 * 4999)
        assert set(r["snapshots"]) == {0.1, 0.5}
    else:
        assert r["failed_at"] == pytest.approx(bad * 1e-4) and r["steps"] == bad
        assert r["max_abs_de"] == pytest.approx(1e-9 * (bad - 1))
        assert r["times"][-1] == pytest.approx(2300 * 1e-4) and r["final"] is None
    assert r["e0"] == pytest.approx(-0.05) and r["mass_drift"] == 0.0
