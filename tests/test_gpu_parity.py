"""GPU parity: the HIP path (through the C ABI) against the FP64 CPU oracle on the same seeded
inputs.  Bars: FP64 1e-12 relative per step on the state; FP32 1e-5 relative on rho and T after
100 steps; derivatives and force coefficients at round-off of their own arithmetic."""
import numpy as np
import pytest

from oracle import dvm as odvm
from oracle import model, spectral
from paper_1403_3746_amd import workloads as W
from tests.gpu_util import field_errors, rel, say

pytestmark = pytest.mark.gpu

SIZES = (8, 12, 16, 24, 32, 48, 64, 96, 128, 192, 256, 384, 512, 768, 1024, 1536, 2048)


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _sim(instances, precision="fp64"):
    from paper_1403_3746_amd.lbfft import Sim
    return Sim(instances, precision)


def _moments(p):
    return lambda f: model.moments(f, p)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("n", SIZES)
def test_derivative_every_line_length(torch_cuda, n, prec):
    # x derivative on an n x 8 grid and y derivative on an 8 x n grid: every FFT instantiation
    rng = np.random.default_rng(n)
    dx = 0.7
    tol = 2e-13 if prec == "fp64" else 3e-6
    for nx, ny, axis in ((n, 8, 0), (8, n, 1)):
        p = W.base_params(dx=dx)
        sim = _sim([(p, W.slab(nx, ny, 0.5))], prec)
        g = rng.normal(size=(ny, nx))
        for order in (1, 2):
            ref = spectral.dx_(g, dx) if axis == 0 else spectral.dy_(g, dx)
            if order == 2:
                ref = spectral.dx_(ref, dx) if axis == 0 else spectral.dy_(ref, dx)
            out = sim.derivative(g, axis, order)
            e = rel(out, ref)
            say(f"derivative n={n} axis={axis} order={order} {prec}: rel err {e:.2e}")
            assert e < tol * (1 + np.log2(n)) / 4
        sim.close()


@pytest.mark.parametrize("grid", [(2, 64), (1, 96), (2, 2048)])
def test_quasi_1d_y_derivative_vanishes(torch_cuda, grid):
    ny, nx = grid
    p = W.base_params()
    sim = _sim([(p, W.slab(nx, ny, 0.5))])
    g = np.random.default_rng(1).normal(size=(ny, nx))
    assert np.abs(sim.derivative(g, 1, 1)).max() == 0.0
    ref = spectral.dx_(g, 1.0)
    assert rel(sim.derivative(g, 0, 1), ref) < 1e-13
    sim.close()


CASES = [dict(), dict(q=-0.004, zeta=0.01, H=0.003), dict(b=3.0, q=0.02)]


@pytest.mark.parametrize("kw", CASES)
@pytest.mark.parametrize("grid", [(64, 64), (48, 96)])
def test_force_coefficients_fp64(torch_cuda, kw, grid):
    ny, nx = grid
    p = W.base_params(**kw)
    ic = W.smooth_random(nx, ny, 3, T0=0.5)
    sim = _sim([(p, ic)])
    f = sim.get_f()
    rho, ux, uy, T = model.moments(f, p)
    Bx, By, C, Cq = model.force_coefficients(rho, ux, uy, T, p)
    gBx, gBy, gC = sim.force_coefficients()
    errs = (rel(gBx, Bx), rel(gBy, By), rel(gC, C + Cq))
    say(f"force {grid} {kw}: {errs}")
    assert max(errs) < 1e-11
    sim.close()


@pytest.mark.parametrize("kw", CASES)
def test_rhs_fp64(torch_cuda, kw):
    ny, nx = 32, 48
    p = W.base_params(**kw)
    ic = W.smooth_random(nx, ny, 5, T0=0.5)
    sim = _sim([(p, ic)])
    f = sim.get_f()
    rng = np.random.default_rng(7)
    f = f * (1 + 0.01 * rng.uniform(-1, 1, f.shape))     # leave equilibrium
    sim.set_f(f)
    R = sim.rhs()
    ref = model.rhs(f, p)
    e = rel(R, ref)
    say(f"rhs {kw}: {e:.2e}")
    assert e < 1e-11
    sim.close()


def test_step_fp64_slab64_every_step(torch_cuda):
    (p, ic), = W.config("slab64")[0]
    sim = _sim([(p, ic)])
    f_ref = model.init_equilibrium(*ic, p)
    assert rel(sim.get_f(), f_ref) < 1e-14
    worst = 0.0
    for n in range(1, 101):
        sim.step(1)
        f_ref = model.rk2_step(f_ref, p)
        errs = field_errors(sim.get_f(), f_ref, _moments(p))
        worst = max(worst, max(errs.values()))
        if n in (1, 10, 100):
            say(f"slab64 fp64 step {n}: {errs}")
        assert max(errs.values()) < 1e-12, (n, errs)
    say(f"slab64 fp64 worst over 100 steps: {worst:.2e}")
    sim.close()


@pytest.mark.parametrize("b", [2.0, 3.0])
def test_step_fp64_nonsquare_with_all_terms(torch_cuda, b):
    # 20 steps with every term of B, C, C_q switched on, b = 2 and b = 3 degrees of freedom
    ny, nx = 96, 64
    p = W.base_params(q=-0.004, zeta=0.01, H=0.003, dx=0.5, b=b)
    ic = W.smooth_random(nx, ny, 11, T0=0.5)
    sim = _sim([(p, ic)])
    f_ref = model.init_equilibrium(*ic, p)
    for n in range(1, 21):
        sim.step(1)
        f_ref = model.rk2_step(f_ref, p)
        errs = field_errors(sim.get_f(), f_ref, _moments(p))
        assert max(errs.values()) < 1e-12, (n, errs)
    say(f"nonsquare fp64 b={b} step 20: {errs}")
    sim.close()


def test_step_fp32_quench_100(torch_cuda):
    n = 128
    p = W.base_params()
    ic = W.quench(n, n, 0.9 * W.T_C, 2000)
    sim = _sim([(p, ic)], "fp32")
    f_ref = model.run(model.init_equilibrium(*ic, p), p, 100)
    sim.step(100)
    errs = field_errors(sim.get_f(), f_ref, _moments(p))
    say(f"quench128 fp32 step 100: {errs}")
    assert errs["rho"] < 1e-5 and errs["T"] < 1e-5
    sim.close()


def test_conservation_and_checkpoint(torch_cuda):
    p = W.base_params(q=-0.004)
    ic = W.smooth_random(64, 64, 13, T0=0.5)
    sim = _sim([(p, ic)])
    c0 = sim.conservation()
    ref = model.conservation(model.init_equilibrium(*ic, p), p)
    say(f"conservation gpu {c0} oracle {ref}")
    assert abs(c0[0] - ref[0]) < 1e-12 * abs(ref[0])
    assert abs(c0[3] - ref[3]) < 1e-11 * abs(ref[3])
    sim.step(5)
    f5 = sim.get_f()
    sim.step(5)
    f10 = sim.get_f()
    c1 = sim.conservation()
    assert abs(c1[0] - c0[0]) < 1e-12 * abs(c0[0])
    assert abs(c1[1] - c0[1]) < 1e-12 * abs(c0[0]) and abs(c1[2] - c0[2]) < 1e-12 * abs(c0[0])
    sim.set_f(f5)
    sim.step(5)
    assert np.array_equal(sim.get_f(), f10)
    sim.close()


def test_nonfinite_state_is_reported(torch_cuda):
    from paper_1403_3746_amd import lbfft
    p = W.base_params()
    sim = _sim([(p, W.slab(32, 32, 0.5))])
    f = sim.get_f()
    f[3, 5, 7] = np.nan
    sim.set_f(f)
    with pytest.raises(lbfft.LBError) as e:
        sim.conservation()
    assert e.value.status == lbfft.LB_E_NONFINITE
    sim.close()


def test_ragged_batch_matches_solo_and_oracle(torch_cuda, monkeypatch):
    # three sizes, four instances, one context: each instance equals its solo run bitwise and the
    # oracle within the FP64 bar after 10 steps.  The launch plan is pinned: separately tuned
    # contexts may pick x-pass plans that round differently.
    monkeypatch.setenv("LBFFT_PPB", "2")
    monkeypatch.setenv("LBFFT_XPOP", "0")
    insts = [(W.base_params(), W.slab(64, 64, 0.52)),
             (W.base_params(), W.quench(96, 96, 0.53, 5)),
             (W.base_params(q=-0.004), W.quench(64, 64, 0.55, 6)),
             (W.base_params(), W.slab(128, 32, 0.5))]
    sim = _sim(insts)
    sim.step(10)
    for k, (p, ic) in enumerate(insts):
        solo = _sim([(p, ic)])
        solo.step(10)
        fb, fs = sim.get_f(k), solo.get_f()
        assert np.array_equal(fb, fs), k
        f_ref = model.run(model.init_equilibrium(*ic, p), p, 10)
        errs = field_errors(fb, f_ref, _moments(p))
        say(f"batch inst {k} {ic[0].shape}: {errs}")
        assert max(errs.values()) < 1e-12
        solo.close()
    sim.close()


def test_step_timed_matches_graph_step(torch_cuda, monkeypatch):
    monkeypatch.setenv("LBFFT_PPB", "2")   # one plan for both contexts
    monkeypatch.setenv("LBFFT_XPOP", "0")
    p = W.base_params()
    ic = W.quench(64, 48, 0.52, 9)
    a, b = _sim([(p, ic)]), _sim([(p, ic)], )
    a.step(4)
    ms = b.step_timed(4)
    assert all(v > 0 for v in ms.values()), ms
    assert np.array_equal(a.get_f(), b.get_f())
    a.close()
    b.close()


def test_fused_xy_passes_match_separate_passes(torch_cuda, monkeypatch):
    # square grids run the x and y macroscopic passes of a stage as one launch; the per-line
    # arithmetic is the same, so the state must agree bit for bit with the separate launches
    p = W.base_params()
    ic = W.quench(96, 96, 0.52, 21)
    monkeypatch.setenv("LBFFT_PPB", "2")   # same x-pass plan for both (no tuning difference)
    monkeypatch.setenv("LBFFT_XPOP", "0")
    for prec in ("fp64", "fp32"):
        monkeypatch.setenv("LBFFT_FUSE_XY", "0")
        sep = _sim([(p, ic)], prec)
        monkeypatch.delenv("LBFFT_FUSE_XY")
        fused = _sim([(p, ic)], prec)
        sep.step(5)
        ms = fused.step_timed(5)
        assert ms["macro_y1"] == 0 and ms["macro_y2"] == 0, ms
        assert all(ms[k] > 0 for k in ms if k not in ("macro_y1", "macro_y2")), ms
        assert np.array_equal(sep.get_f(), fused.get_f()), prec
        sep.close()
        fused.close()


def test_conservation_history_matches_oracle(torch_cuda):
    p = W.base_params(q=-0.004, hist=20)
    ic = W.smooth_random(48, 32, 17, T0=0.5)
    sim = _sim([(p, ic)])
    c0 = sim.conservation()
    sim.step(10)
    first, h = sim.history()
    assert first == 0 and h.shape == (10, 4)
    assert np.array_equal(h[0], c0)
    f = model.init_equilibrium(*ic, p)
    for n in range(10):
        ref = model.conservation(f, p)
        assert abs(h[n, 0] - ref[0]) < 1e-12 * abs(ref[0])
        assert abs(h[n, 1] - ref[1]) < 1e-12 * abs(ref[0]) and abs(h[n, 2] - ref[2]) < 1e-12 * abs(ref[0])
        assert abs(h[n, 3] - ref[3]) < 1e-11 * abs(ref[3])
        f = model.rk2_step(f, p)
    say(f"history mass drift over 10 steps: {h[-1, 0] - h[0, 0]:.3e}")
    sim.close()


def test_conservation_history_ring_wraps(torch_cuda):
    insts = [(W.base_params(hist=4), W.slab(32, 32, 0.5)), (W.base_params(), W.slab(32, 32, 0.52))]
    sim = _sim(insts)
    sim.step(10)
    first, h = sim.history(0)
    assert first == 6 and h.shape == (4, 4)
    from paper_1403_3746_amd import lbfft
    with pytest.raises(lbfft.LBError) as e:
        sim.history(1)
    assert e.value.status == lbfft.LB_E_STATE
    sim.close()


@pytest.mark.parametrize("ppb", ["1", "2", "4"])
def test_full_step_square_sizes_of_three_times_pow2(torch_cuda, monkeypatch, ppb):
    # one RK2 step of square 3*2^a grids (radix-12 lines, fused x+y passes, every x-pass plan)
    # against the oracle; the derivative test covers these lengths in the macroscopic passes only
    monkeypatch.setenv("LBFFT_PPB", ppb)
    for n in (24, 96, 192, 384):
        p = W.base_params(q=-0.004, zeta=1e-3)
        ic = W.smooth_random(n, n, 100 + n, T0=0.52)
        sim = _sim([(p, ic)])
        f = model.rk2_step(model.init_equilibrium(*ic, p), p)
        sim.step(1)
        g = sim.get_f()
        err = np.abs(g - f).max() / np.abs(f).max()
        say(f"full step {n}x{n} pops/block {ppb}: rel err {err:.2e}")
        assert err < 1e-12, (n, ppb, err)
        sim.close()


@pytest.mark.parametrize("prec,ypop,ymac", [("fp64", "0", "0"), ("fp32", "0", "0"), ("fp32", "1", "0"),
                                           ("fp32", "2", "2")])
def test_step_long_columns(torch_cuda, monkeypatch, prec, ypop, ymac):
    # tall grids: y lines of 768..2048 points (narrow column-pair tiles, blocks in job-major
    # order), with the last tile partly empty where nx/2 is not a multiple of the tile width; in
    # FP32 with each y-pass plan: default, wide population y tiles, radix-16 y passes
    monkeypatch.setenv("LBFFT_YPOP", ypop)
    monkeypatch.setenv("LBFFT_YMAC", ymac)
    tol = 1e-12 if prec == "fp64" else 2e-6
    for ny, nx in ((768, 24), (1024, 24), (1536, 12), (2048, 12)):
        p = W.base_params(q=-0.004, zeta=1e-3)
        ic = W.smooth_random(nx, ny, 7 + ny, T0=0.52)
        sim = _sim([(p, ic)], prec)
        if prec == "fp32" and ny in (1024, 2048):
            assert sim.plan(0)["pop_y_plan"] == int(ypop) and sim.plan(0)["macro_y_plan"] == int(ymac)
        f_ref = model.init_equilibrium(*ic, p)
        for _ in range(3):
            f_ref = model.rk2_step(f_ref, p)
        sim.step(3)
        errs = field_errors(sim.get_f(), f_ref, _moments(p))
        say(f"long columns {nx}x{ny} {prec} y plans {ypop}/{ymac} step 3: {errs}")
        assert max(errs.values()) < tol, (ny, nx, errs)
        sim.close()


@pytest.mark.parametrize("prec,ppb", [("fp64", "2"), ("fp32", "1"), ("fp32", "2"), ("fp32", "4")])
def test_step_long_rows(torch_cuda, monkeypatch, prec, ppb):
    # wide grids: x lines of 768 and 1536 points (radix-12 plans, the FP32 ones with all their
    # twiddles preloaded) through the population x pass in each plan, three steps
    monkeypatch.setenv("LBFFT_PPB", ppb)
    tol = 1e-12 if prec == "fp64" else 2e-6
    for nx, ny in ((768, 24), (1536, 12)):
        p = W.base_params(q=-0.004, zeta=1e-3)
        ic = W.smooth_random(nx, ny, 11 + nx, T0=0.52)
        sim = _sim([(p, ic)], prec)
        assert sim.plan(0)["pops_per_block_x"] == int(ppb)
        f_ref = model.init_equilibrium(*ic, p)
        for _ in range(3):
            f_ref = model.rk2_step(f_ref, p)
        sim.step(3)
        errs = field_errors(sim.get_f(), f_ref, _moments(p))
        say(f"long rows {nx}x{ny} {prec} pops/block {ppb} step 3: {errs}")
        assert max(errs.values()) < tol, (nx, ny, errs)
        sim.close()


def test_multi_step_graph_matches_single_step_replays(torch_cuda, monkeypatch):
    # a single size class steps through a graph of several steps while enough remain; its state
    # must equal that of one-step replays bit for bit, history included (37 = 2 * 16 + 5)
    monkeypatch.setenv("LBFFT_PPB", "2")   # one plan for both contexts
    monkeypatch.setenv("LBFFT_XPOP", "0")
    p = W.base_params(hist=64)
    ic = W.quench(64, 64, 0.9 * W.T_C, 11)
    out = {}
    for k in ("1", "16"):
        monkeypatch.setenv("LBFFT_GRAPH_STEPS", k)
        sim = _sim([(p, ic)], "fp32")
        sim.step(37)
        out[k] = (sim.get_f(), sim.history())
        sim.close()
    assert np.array_equal(out["1"][0], out["16"][0])
    assert out["1"][1][0] == out["16"][1][0] == 0
    assert np.array_equal(out["1"][1][1], out["16"][1][1]) and out["16"][1][1].shape == (37, 4)


def test_ragged_multi_step_graph_matches_single_step_replays(torch_cuda, monkeypatch):
    # a batch of several size classes replays a graph of several steps whose class branches join
    # only at its end; states and histories must equal one-step replays bit for bit
    monkeypatch.setenv("LBFFT_PPB", "2")
    monkeypatch.setenv("LBFFT_XPOP", "0")
    insts = [(W.base_params(hist=64), W.quench(64, 64, 0.9 * W.T_C, 12)),
             (W.base_params(), W.slab(96, 96, 0.52)),
             (W.base_params(hist=40), W.quench(128, 32, 0.53, 13)),
             (W.base_params(), W.quench(64, 64, 0.51, 14))]
    out = {}
    for k in ("1", "16"):
        monkeypatch.setenv("LBFFT_GRAPH_STEPS", k)
        sim = _sim(insts, "fp32")
        assert sim.plan(0)["size_classes"] == 3
        sim.step(37)
        out[k] = ([sim.get_f(i) for i in range(len(insts))], sim.history(0), sim.history(2))
        sim.close()
    for i in range(len(insts)):
        assert np.array_equal(out["1"][0][i], out["16"][0][i]), i
    for h in (1, 2):
        assert out["1"][h][0] == out["16"][h][0]
        assert np.array_equal(out["1"][h][1], out["16"][h][1])
    assert out["16"][1][1].shape == (37, 4) and out["16"][2][0] == 0


@pytest.mark.parametrize("ymac", ["0", "2"])
def test_fused_square_1024_fp32_every_y_plan(torch_cuda, monkeypatch, ymac):
    # a square grid of 1024-point lines: the fused x + y macroscopic pass with the default and the
    # radix-16 plan (its x tiles then hold 16 elements per thread too), against the oracle
    monkeypatch.setenv("LBFFT_YMAC", ymac)
    monkeypatch.setenv("LBFFT_YPOP", "2" if ymac == "2" else "0")
    n = 1024
    p = W.base_params(q=-0.004, zeta=1e-3)
    ic = W.smooth_random(n, n, 77, T0=0.52)
    from tests.oracle_pool import oracle_workers
    spectral.set_workers(oracle_workers())
    f = model.rk2_step(model.init_equilibrium(*ic, p), p)
    spectral.set_workers(1)
    sim = _sim([(p, ic)], "fp32")
    assert sim.plan(0)["macro_y_plan"] == int(ymac)
    sim.step(1)
    errs = field_errors(sim.get_f(), f, _moments(p))
    say(f"square 1024 fp32 macro y plan {ymac}: {errs}")
    assert errs["rho"] < 2e-6 and errs["T"] < 2e-6
    sim.close()


@pytest.mark.parametrize("ypop,ymac", [("2", "0"), ("0", "2"), ("2", "2")])
def test_fp32_long_radix_plans_of_three_times_pow2(torch_cuda, monkeypatch, ypop, ymac):
    # the FP32 long-radix plans of 3*2^a lines (24 elements per thread: a radix-24 pass, then
    # radix 8) in the population y pass and in the macroscopic y pass -- fused with the x pass on
    # square grids, separate on the others -- two steps against the oracle
    monkeypatch.setenv("LBFFT_YPOP", ypop)
    monkeypatch.setenv("LBFFT_YMAC", ymac)
    for nx, n in ((96, 96), (192, 192), (384, 384), (64, 192), (256, 96)):
        p = W.base_params(q=-0.004, zeta=1e-3)
        ic = W.smooth_random(nx, n, 700 + nx + n, T0=0.52)
        sim = _sim([(p, ic)], "fp32")
        assert sim.plan(0)["pop_y_plan"] == int(ypop) and sim.plan(0)["macro_y_plan"] == int(ymac)
        f = model.init_equilibrium(*ic, p)
        for _ in range(2):
            f = model.rk2_step(f, p)
        sim.step(2)
        errs = field_errors(sim.get_f(), f, _moments(p))
        say(f"fp32 long radix {nx}x{n} y plans {ypop}/{ymac}: {errs}")
        assert max(errs.values()) < 2e-6, (nx, n, ypop, ymac, errs)
        sim.close()


@pytest.mark.parametrize("ppb", ["1", "2", "4"])
def test_fp32_x_pass_four_elements_per_thread(torch_cuda, monkeypatch, ppb):
    # the FP32 x population pass plan with 4 elements per thread (x lines of 128, 256 and 512
    # points spread over twice the threads: one or two waves per line) in each populations-per-
    # block setting, including a missing second row, two steps against the oracle
    monkeypatch.setenv("LBFFT_PPB", ppb)
    monkeypatch.setenv("LBFFT_XPOP", "1")
    for ny, nx in ((24, 128), (16, 256), (8, 512), (1, 128), (2, 256)):
        p = W.base_params(q=-0.004, zeta=1e-3)
        ic = W.smooth_random(nx, ny, 500 + nx + ny, T0=0.52) if ny > 2 else W.slab(nx, ny, 0.52)
        sim = _sim([(p, ic)], "fp32")
        assert sim.plan(0)["pops_per_block_x"] == int(ppb) and sim.plan(0)["pop_x_plan"] == 1
        f = model.init_equilibrium(*ic, p)
        for _ in range(2):
            f = model.rk2_step(f, p)
        sim.step(2)
        errs = field_errors(sim.get_f(), f, _moments(p))
        say(f"fp32 x pass 4/thread, plan {ppb}, {nx}x{ny}: {errs}")
        assert max(errs.values()) < 2e-6, (ppb, nx, ny, errs)
        sim.close()


@pytest.mark.parametrize("ppb", ["1", "2", "4"])
def test_full_step_every_x_pass_plan(torch_cuda, monkeypatch, ppb):
    # two RK2 steps (both stages: base folded, then read per cell) with each x-pass plan, on grids
    # that give its blocks one or several lines, lines of one or several waves, 4, 8 or 12
    # elements per thread and a missing second row (ny = 1), against the oracle
    monkeypatch.setenv("LBFFT_PPB", ppb)
    for ny, nx in ((64, 64), (24, 128), (2, 512), (1, 96), (8, 32), (8, 1024), (8, 2048)):
        p = W.base_params(q=-0.004, zeta=1e-3)
        ic = W.smooth_random(nx, ny, 300 + nx + ny, T0=0.52) if ny > 2 else W.slab(nx, ny, 0.52)
        sim = _sim([(p, ic)])
        assert sim.plan(0)["pops_per_block_x"] == int(ppb)
        f = model.init_equilibrium(*ic, p)
        for _ in range(2):
            f = model.rk2_step(f, p)
        sim.step(2)
        err = np.abs(sim.get_f() - f).max() / np.abs(f).max()
        say(f"x-pass plan {ppb}, {nx}x{ny}: rel err {err:.2e}")
        assert err < 1e-12, (ppb, nx, ny, err)
        sim.close()
