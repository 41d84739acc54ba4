"""Liquid-vapour coexistence curve driver (Sec. 3.1).

A quasi-one-dimensional periodic slab (liquid in the middle half, vapour outside) is stepped with
the library's RK2 step until its bulk densities settle; the settled (T, rho_v, rho_l) is recorded,
the temperature is lowered by a fixed amount -- the state is restarted from the equilibrium of
its current density and velocity at the new uniform temperature -- and the run continues.  The
paper gives the set-up (512 x 2 grid, rho_v = 0.955, rho_l = 1.045, T0 = 0.9975, tau = 1e-4,
dt = 5e-5, dx = 0.02, K = 1e-5, H = zeta = 0, q = -0.004, b = 2, the van der Waals fluid with
a = 9/8, b_w = 1/3) but not the step-down rule, what counts as settled, or how the temperature is
held: in this closed system the latent heat released while the phases separate raises the
temperature again after each step-down.  Here a temperature is settled when the bulk densities,
averaged over consecutive windows of checks, change by less than `tol` (relative to
rho_l - rho_v) between windows; with `hold` (the default) the state is also restarted at the set
temperature at every check -- f = f^eq(rho, u, T_set) from its own density and velocity -- so
the run settles at that temperature (the mean temperature reached since the last check is
recorded as well).

Everything runs through the HIP library (`lbfft.Sim`); the host only reads the moments at each
check and rewrites the state at each step-down.
"""
import argparse
import json
import sys
import time

import numpy as np

from . import lbfft

# Sec. 3.1 parameters; the fluid is the paper's own van der Waals EOS (T_c = rho_c = 1).
PAPER_PARAMS = dict(dx=0.02, dt=5e-5, tau=1e-4, K=1e-5, H=0.0, zeta=0.0, q=-0.004, b=2.0,
                    a=9.0 / 8.0, bw=1.0 / 3.0)
# The paper takes the D2V16 ring speeds from Kataoka and Tsutahara without printing them.  For
# T near 1 the default rings (1, 0.5, 2, 1) are scaled by 1.15: the smallest scale that keeps every
# f^eq above -1.2e-4 rho over T in [0.75, 1], |u| <= 0.05.
COEX_DVM = dict(va=1.15, vb=0.575, vc=2.3, vd=1.15, eta0=2.5)


def scaled_rings(scale, eta0=2.5):
    """The default ring speeds (1, 0.5, 2, 1) times `scale` (COEX_DVM is scale 1.15)."""
    return dict(va=scale, vb=0.5 * scale, vc=2.0 * scale, vd=scale, eta0=eta0)


def slab(nx=512, ny=2, rho_v=0.955, rho_l=1.045, T0=0.9975):
    """Sec. 3.1 initial state: vapour for j <= nx/4 and j > 3nx/4, liquid between, at rest."""
    j = np.arange(nx)
    prof = np.where((j > nx // 4) & (j <= 3 * nx // 4), rho_l, rho_v).astype(np.float64)
    rho = np.broadcast_to(prof[None, :], (ny, nx)).copy()
    z = np.zeros((ny, nx))
    return rho, z.copy(), z.copy(), np.full((ny, nx), float(T0))


def bulk_densities(rho, frac=0.1):
    """Vapour and liquid bulk densities: means of the lowest and highest `frac` of the column
    averages of rho (away from the interfaces, which hold few cells)."""
    prof = np.sort(rho.mean(axis=0))
    k = max(1, int(frac * prof.size))
    return float(prof[:k].mean()), float(prof[-k:].mean())


class Settler:
    """Plateau detector over checks: windows of `window` checks; settled once the window means of
    rho_v and rho_l both move by less than tol * (rho_l - rho_v) from one window to the next and
    the largest flow speed seen in the last window is below u_tol (a sloshing slab can pass
    through the same densities twice)."""

    def __init__(self, window=5, tol=2e-4, u_tol=1e-2):
        self.window, self.tol, self.u_tol = window, tol, u_tol
        self.samples, self.means, self.umax = [], [], []

    def add(self, rho_v, rho_l, u_max=0.0):
        self.samples.append((rho_v, rho_l))
        self.umax.append(u_max)
        if len(self.samples) % self.window:
            return False
        m = np.mean(self.samples[-self.window:], axis=0)
        self.means.append(m)
        if len(self.means) < 2 or max(self.umax[-self.window:]) >= self.u_tol:
            return False
        d = np.abs(self.means[-1] - self.means[-2])
        return bool(np.all(d < self.tol * max(m[1] - m[0], 1e-12)))

    def estimate(self):
        return tuple(self.means[-1]) if self.means else self.samples[-1]


def run(temperatures, precision="fp64", nx=512, ny=2, check=2000, window=5, tol=2e-4,
        max_steps=2_000_000, hold=True, log=None, params=None, dvm=None, ic=None):
    """Step the Sec. 3.1 slab through the given temperatures (the first is the initial one).
    Returns one record per temperature: T (the set value), T_mean (mean temperature of the
    state at the last check, before any restart), rho_v, rho_l (window means), steps, settled
    (False if max_steps ran out), u_max, seconds.  `ic` replaces the Sec. 3.1 slab by a given
    (rho, ux, uy, T) state."""
    p = dict(PAPER_PARAMS, **(params or {}))
    state = ic if ic is not None else slab(nx, ny, T0=temperatures[0])
    sim = lbfft.Sim([(p, state)], precision, dvm=dvm or COEX_DVM)
    out = []
    try:
        for k, T in enumerate(temperatures):
            if k > 0:
                rho, ux, uy, _ = sim.moments()
                sim.set_moments(rho, ux, uy, np.full_like(rho, T))
            st = Settler(window, tol)
            t0, n, settled = time.perf_counter(), 0, False
            while n < max_steps:
                sim.step(check)
                n += check
                rho, ux, uy, TT = sim.moments()
                if not np.all(np.isfinite(rho)):
                    raise RuntimeError(f"non-finite state at T = {T} after {n} steps")
                rv, rl = bulk_densities(rho)
                settled = st.add(rv, rl, float(np.abs(ux).max()))
                if log:
                    log(f"T={T:.5f} step {n} rho_v {rv:.6f} rho_l {rl:.6f} "
                        f"T_mean {TT.mean():.6f} T_range {TT.max() - TT.min():.2e} "
                        f"u_max {np.abs(ux).max():.2e}")
                if settled:
                    break
                if hold:
                    sim.set_moments(rho, ux, uy, np.full_like(rho, T))
            rv, rl = st.estimate()
            out.append(dict(T=T, T_mean=float(TT.mean()), rho_v=rv, rho_l=rl, steps=n,
                            settled=settled, u_max=float(np.abs(ux).max()),
                            seconds=time.perf_counter() - t0))
    finally:
        sim.close()
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--temperatures", type=float, nargs="+",
                    default=[0.9975, 0.99, 0.98, 0.97, 0.95, 0.93, 0.9, 0.87, 0.85, 0.82, 0.8])
    ap.add_argument("--precision", default="fp64", choices=("fp64", "fp32"))
    ap.add_argument("--check", type=int, default=2000)
    ap.add_argument("--window", type=int, default=5)
    ap.add_argument("--tol", type=float, default=2e-4)
    ap.add_argument("--max-steps", type=int, default=2_000_000)
    ap.add_argument("--no-hold", action="store_true",
                    help="do not restart at the set temperature at every check")
    ap.add_argument("--K", type=float, default=PAPER_PARAMS["K"],
                    help="surface-tension coefficient (the Sec. 3.1 value by default)")
    ap.add_argument("--nx", type=int, default=512)
    ap.add_argument("--dx", type=float, default=PAPER_PARAMS["dx"],
                    help="grid spacing (with --nx: the same slab at another resolution)")
    ap.add_argument("--ring-scale", type=float, default=1.15,
                    help="ring speeds (1, 0.5, 2, 1) times this factor (the paper does not print them)")
    ap.add_argument("--json", help="write the records here")
    a = ap.parse_args(argv)
    recs = run(a.temperatures, a.precision, nx=a.nx, check=a.check, window=a.window, tol=a.tol,
               max_steps=a.max_steps, hold=not a.no_hold, params=dict(K=a.K, dx=a.dx),
               dvm=scaled_rings(a.ring_scale), log=lambda s: print(s, flush=True))
    for r in recs:
        print(json.dumps(r), flush=True)
    if a.json:
        json.dump(recs, open(a.json, "w"), indent=1)


if __name__ == "__main__":
    sys.exit(main())
