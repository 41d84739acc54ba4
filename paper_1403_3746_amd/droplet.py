"""Large deformation of a rectangular droplet under surface tension, and the spurious velocity
(Sec. 3.3).

A 118 x 14 (cells) liquid rectangle (rho_l = 1.462) in vapour (rho_v = 0.579) relaxes towards a
circle at the fixed temperature T = 0.95, with dx = dy = 0.01, tau = 5 dt = 5e-4, K = 1e-5,
q = -0.05 and the paper's van der Waals fluid.  The paper does not give the domain size; here it
is 192 x 192 cells, the droplet centred (37 cells of vapour beyond each end).  "T fixed" is read
as the run's strong heat conduction (q = -0.05), which keeps the temperature within a few 1e-3 of
0.95 by itself; `run` records the temperature range to show it.  (Restarting the state at
T = 0.95 every `hold_every` steps, f = f^eq(rho, u, 0.95), is available but destabilises this
run: it removes the non-equilibrium part of f, which carries the viscous stress.)  At every check
`run` records the largest flow speed (the spurious velocity u_max^s once the droplet has
settled), the droplet's aspect ratio from the second moments of its liquid excess, its area and
the temperature range.
"""
import argparse
import json
import sys
import time

import numpy as np

from . import lbfft
from .coexistence import COEX_DVM

PAPER_PARAMS = dict(dx=0.01, dt=1e-4, tau=5e-4, K=1e-5, H=0.0, zeta=0.0, q=-0.05, b=2.0,
                    a=9.0 / 8.0, bw=1.0 / 3.0)
RHO_L, RHO_V, T_FIX = 1.462, 0.579, 0.95


def initial(n=192, length=118, height=14, width=1.0):
    """The rectangle centred in an n x n box, edges smoothed over `width` cells (tanh)."""
    c = (n - 1) / 2.0
    j = np.arange(n) - c
    sx = 0.5 * (1.0 + np.tanh((length / 2.0 - np.abs(j)) / width))
    sy = 0.5 * (1.0 + np.tanh((height / 2.0 - np.abs(j)) / width))
    rho = RHO_V + (RHO_L - RHO_V) * np.outer(sy, sx)
    z = np.zeros((n, n))
    return rho, z.copy(), z.copy(), np.full((n, n), T_FIX)


def shape(rho):
    """(aspect ratio >= 1, liquid area in cells) from the second moments of the liquid excess
    w = clip((rho - rho_mid) / (rho_l - rho_v) + 1/2, 0, 1) about its centroid."""
    w = np.clip((rho - 0.5 * (RHO_L + RHO_V)) / (RHO_L - RHO_V) + 0.5, 0.0, 1.0)
    ny, nx = rho.shape
    y, x = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    m = w.sum()
    cx, cy = (w * x).sum() / m, (w * y).sum() / m
    ixx, iyy, ixy = (w * (x - cx) ** 2).sum() / m, (w * (y - cy) ** 2).sum() / m, (w * (x - cx) * (y - cy)).sum() / m
    ev = np.linalg.eigvalsh(np.array([[ixx, ixy], [ixy, iyy]]))
    return float(np.sqrt(ev[1] / max(ev[0], 1e-300))), float(m)


def run(t_end=100.0, precision="fp64", n=192, check_every=2000, hold_every=0, params=None,
        dvm=None, log=None, length=118, height=14):
    """Returns dict(times, u_max, aspect, area, T_range, steps, failed_at, seconds); hold_every > 0
    restarts the state at T = 0.95 every that many steps."""
    p = dict(PAPER_PARAMS, **(params or {}))
    steps = int(round(t_end / p["dt"]))
    sim = lbfft.Sim([(p, initial(n, length, height))], precision, dvm=dvm or COEX_DVM)
    times, umax, aspect, area, trange = [], [], [], [], []
    done, t0, failed_at = 0, time.perf_counter(), None
    interval = hold_every if hold_every > 0 else check_every
    try:
        rho, ux, uy, _ = sim.moments()
        a, m = shape(rho)
        times.append(0.0), umax.append(0.0), aspect.append(a), area.append(m), trange.append(0.0)
        while done < steps:
            k = min(interval, steps - done)
            sim.step(k)
            done += k
            rho, ux, uy, T = sim.moments()
            if not np.all(np.isfinite(rho)):
                failed_at = done * p["dt"]
                break
            if hold_every > 0:
                sim.set_moments(rho, ux, uy, np.full_like(rho, T_FIX))
            if done % check_every == 0 or done == steps:
                a, m = shape(rho)
                times.append(done * p["dt"])
                umax.append(float(np.hypot(ux, uy).max()))
                aspect.append(a)
                area.append(m)
                trange.append(float(T.max() - T.min()))
                if log:
                    log(f"t {done * p['dt']:.2f} u_max {umax[-1]:.3e} aspect {a:.4f} area {m:.1f} "
                        f"T range {T.max() - T.min():.2e} {time.perf_counter() - t0:.0f} s")
    finally:
        sim.close()
    return dict(times=times, u_max=umax, aspect=aspect, area=area, T_range=trange, steps=done,
                failed_at=failed_at,
                seconds=time.perf_counter() - t0)


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--t-end", type=float, default=100.0)
    ap.add_argument("--n", type=int, default=192)
    ap.add_argument("--precision", default="fp64", choices=("fp64", "fp32"))
    ap.add_argument("--hold-every", type=int, default=0)
    ap.add_argument("--check-every", type=int, default=2000)
    ap.add_argument("--length", type=int, default=118, help="droplet length in cells")
    ap.add_argument("--height", type=int, default=14, help="droplet height in cells")
    ap.add_argument("--json", help="write the histories here")
    a = ap.parse_args(argv)
    r = run(a.t_end, a.precision, a.n, a.check_every, a.hold_every, log=lambda s: print(s, flush=True),
            length=a.length, height=a.height)
    print(json.dumps({k: r[k] for k in ("steps", "failed_at", "seconds")}), flush=True)
    if a.json:
        json.dump(r, open(a.json, "w"))


if __name__ == "__main__":
    sys.exit(main())
