"""Host logic of the coexistence-curve driver (Sec. 3.1), without a GPU: the initial slab, the
bulk-density estimate, the plateau detector, and the step / check / restart loop run against a
stand-in simulator."""
import numpy as np
import pytest

from paper_1403_3746_amd import coexistence as cx


def test_slab_matches_section_3_1_layout():
    rho, ux, uy, T = cx.slab(512, 2)
    j = np.arange(512)
    liquid = (j > 128) & (j <= 384)
    assert rho.shape == (2, 512) and np.all(rho[:, liquid] == 1.045) and np.all(rho[:, ~liquid] == 0.955)
    assert liquid.sum() == 256 and np.all(ux == 0) and np.all(uy == 0) and np.all(T == 0.9975)


def test_bulk_densities_ignore_the_interfaces():
    x = np.arange(512)
    prof = 1.0 + 0.6 * np.tanh((128 - np.abs(x - 256)) / 3.0)   # liquid 1.6, vapour 0.4
    rv, rl = cx.bulk_densities(np.vstack([prof, prof]))
    assert abs(rv - 0.4) < 1e-6 and abs(rl - 1.6) < 1e-6


def test_settler_waits_for_two_quiet_windows():
    s = cx.Settler(window=3, tol=1e-3)
    # drifting: window means move by 0.01 per window > tol * 1.2
    hits = [s.add(0.4 - 0.01 * k / 3, 1.6) for k in range(12)]
    assert not any(hits)
    s = cx.Settler(window=3, tol=1e-3)
    hits = [s.add(0.4 + 1e-6 * (-1) ** k, 1.6) for k in range(6)]
    assert hits == [False] * 5 + [True]
    assert abs(s.estimate()[0] - 0.4) < 1e-5 and abs(s.estimate()[1] - 1.6) < 1e-12
    # still flowing: no plateau however quiet the densities
    s = cx.Settler(window=3, tol=1e-3, u_tol=1e-2)
    assert not any(s.add(0.4, 1.6, 2e-2) for k in range(9))


class FakeSim:
    """Relaxes the bulk densities of a two-phase profile toward targets that depend on the last
    temperature written by set_moments; records the calls."""
    calls = []

    def __init__(self, instances, precision, dvm=None):
        (p, (rho, ux, uy, T)), = instances
        self.rho, self.ux, self.uy, self.T = rho.copy(), ux.copy(), uy.copy(), T.copy()
        FakeSim.calls = [("init", float(T.mean()), dvm)]

    def step(self, n):
        target_v, target_l = 0.4 + 0.2 * (self.T.mean() - 0.9), 1.6 - 0.2 * (self.T.mean() - 0.9)
        j = np.arange(self.rho.shape[1])
        liquid = (j > self.rho.shape[1] // 4) & (j <= 3 * self.rho.shape[1] // 4)
        goal = np.where(liquid, target_l, target_v)[None, :]
        self.rho = goal + (self.rho - goal) * 0.5 ** (n / 1000.0)
        self.T = self.T + 1e-3   # latent heat: the temperature creeps up between checks
        FakeSim.calls.append(("step", n))

    def moments(self, inst=0):
        return self.rho.copy(), self.ux.copy(), self.uy.copy(), self.T.copy()

    def set_moments(self, rho, ux, uy, T, inst=0):
        self.rho, self.T = np.array(rho), np.array(T)
        FakeSim.calls.append(("set", float(np.mean(T))))

    def close(self):
        FakeSim.calls.append(("close",))


@pytest.mark.parametrize("hold", [True, False])
def test_run_schedule_with_stand_in(monkeypatch, hold):
    monkeypatch.setattr(cx.lbfft, "Sim", FakeSim)
    recs = cx.run([0.95, 0.9], nx=64, ny=2, check=1000, window=2, tol=1e-3, max_steps=200000, hold=hold)
    assert [r["T"] for r in recs] == [0.95, 0.9]
    assert all(r["settled"] for r in recs)
    sets = [c[1] for c in FakeSim.calls if c[0] == "set"]
    assert FakeSim.calls[0][0] == "init" and FakeSim.calls[-1] == ("close",)
    assert FakeSim.calls[0][2] == cx.COEX_DVM
    if hold:
        # every check that does not settle restarts at the set temperature
        assert set(np.round(sets, 12)) == {0.95, 0.9}
        assert abs(recs[1]["T_mean"] - 0.9 - 1e-3) < 1e-9
    else:
        assert sets == pytest.approx([0.9])   # only the step-down
        assert recs[1]["T_mean"] > 0.9 + 2e-3
    for r in recs:
        assert r["rho_l"] > r["rho_v"] and r["steps"] % 1000 == 0


def test_scaled_rings_match_the_default_set():
    from paper_1403_3746_amd import coexistence as C
    assert C.scaled_rings(1.15) == C.COEX_DVM
    d = C.scaled_rings(2.0)
    assert (d["va"], d["vb"], d["vc"], d["vd"], d["eta0"]) == (2.0, 1.0, 4.0, 2.0, 2.5)
