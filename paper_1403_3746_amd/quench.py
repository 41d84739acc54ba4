"""Thermal phase separation after a quench, with the total-energy history (Sec. 3.2).

A 128 x 128 periodic fluid at rest, rho = 1 + (noise of amplitude 0.001), T = 0.9, of the paper's
van der Waals fluid (a = 9/8, b_w = 1/3, T_c = 1), is stepped to t = 200 with tau = 1e-4,
dt = 1e-4, dx = dy = 1/256, K = 5e-6.  The paper leaves H, zeta, q and b unstated for this run;
they take the model's plain values H = zeta = q = 0, b = 2.  The library records the four
FP64 grid integrals (mass, momentum, e_T) of every step on the GPU (conservation history); the
driver reads them back in chunks and reports |e_T(t) - e_T(0)|, the quantity the paper plots,
with density snapshots at the times it shows (t = 1, 2, 25, 200).
"""
import argparse
import json
import sys
import time

import numpy as np

from . import lbfft
from .coexistence import COEX_DVM

PAPER_PARAMS = dict(dx=1.0 / 256.0, dt=1e-4, tau=1e-4, K=5e-6, H=0.0, zeta=0.0, q=0.0, b=2.0,
                    a=9.0 / 8.0, bw=1.0 / 3.0)
# the ring speeds used for T near 1 (see coexistence.COEX_DVM)
QUENCH_DVM = COEX_DVM


def initial(n=128, T=0.9, amp=1e-3, seed=1403):
    """rho = 1 + amp U(-1, 1) i.i.d. per cell, u = 0, uniform T."""
    rng = np.random.default_rng(seed)
    rho = 1.0 + amp * rng.uniform(-1.0, 1.0, (n, n))
    z = np.zeros((n, n))
    return rho, z.copy(), z.copy(), np.full((n, n), float(T))


def snapshot_stats(rho):
    """Summary of a density pattern: extremes, liquid area fraction (rho > 1) and the mean
    wavenumber (in units of 2 pi / L) of the structure factor, whose inverse tracks domain size."""
    d = rho - rho.mean()
    S = np.abs(np.fft.fft2(d)) ** 2
    n = rho.shape[0]
    k = np.fft.fftfreq(n, 1.0 / n)
    K = np.hypot(*np.meshgrid(k, k, indexing="ij"))
    S[0, 0] = 0.0
    kmean = float((K * S).sum() / max(S.sum(), 1e-300))
    return dict(rho_min=float(rho.min()), rho_max=float(rho.max()),
                liquid_fraction=float((rho > 1.0).mean()), k_mean=kmean)


def run(t_end=200.0, precision="fp64", n=128, chunk=100_000, every=100, snap_times=(1, 2, 25, 200),
        params=None, dvm=None, seed=1403, log=None):
    """Returns dict(times, e_T (sampled every `every` steps), max_abs_de (over every finite
    step), mass_drift, snapshots {t: stats}, rho {t: field}, steps (completed), failed_at (time of
    the first non-finite integral, or None), seconds)."""
    p = dict(PAPER_PARAMS, **(params or {}))
    steps = int(round(t_end / p["dt"]))
    chunk = min(chunk, steps)
    p["hist"] = chunk
    sim = lbfft.Sim([(p, initial(n, seed=seed))], precision, dvm=dvm or QUENCH_DVM)
    snap_steps = {int(round(t / p["dt"])): t for t in snap_times if t <= t_end}
    times, eT, max_de, e0, m0, mass_drift = [], [], 0.0, None, None, 0.0
    snaps, fields = {}, {}
    done, t0, failed_at, c = 0, time.perf_counter(), None, None
    try:
        while done < steps:
            # stop at the next snapshot or chunk boundary
            nxt = min([s for s in snap_steps if s > done] + [done + chunk, steps])
            sim.step(nxt - done)
            first, h = sim.history(max_entries=nxt - done, allow_nonfinite=True)
            assert first == done and len(h) == nxt - done, (first, done, len(h))
            bad = np.flatnonzero(~np.all(np.isfinite(h), axis=1))
            if bad.size:
                failed_at = (done + int(bad[0])) * p["dt"]
                h = h[: bad[0]]
                nxt = done + len(h)
            if len(h):
                if e0 is None:
                    e0, m0 = h[0, 3], h[0, 0]
                max_de = max(max_de, float(np.abs(h[:, 3] - e0).max()))
                mass_drift = max(mass_drift, float(np.abs(h[:, 0] - m0).max()))
                for j in range((-done) % every, len(h), every):
                    times.append((done + j) * p["dt"])
                    eT.append(float(h[j, 3]))
            done = nxt
            if failed_at is not None:
                if log:
                    log(f"non-finite state from t {failed_at:.4f}: stopping")
                break
            if done in snap_steps:
                rho = sim.moments()[0]
                t = snap_steps[done]
                snaps[t] = snapshot_stats(rho)
                fields[t] = rho
            if log:
                log(f"step {done} t {done * p['dt']:.2f} max|de_T| {max_de:.3e} "
                    f"mass drift {mass_drift:.2e} {time.perf_counter() - t0:.1f} s")
        if failed_at is None:
            c = sim.conservation()
    finally:
        sim.close()
    return dict(times=times, e_T=eT, e0=None if e0 is None else float(e0), max_abs_de=max_de, mass_drift=mass_drift,
                final=None if c is None else c.tolist(), snapshots=snaps, rho=fields, steps=done,
                failed_at=failed_at, seconds=time.perf_counter() - t0)


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--t-end", type=float, default=200.0)
    ap.add_argument("--precision", default="fp64", choices=("fp64", "fp32"))
    ap.add_argument("--every", type=int, default=1000, help="keep e_T every this many steps")
    ap.add_argument("--json", help="write the summary (history, snapshot statistics) here")
    ap.add_argument("--npz", help="write the density snapshots here")
    ap.add_argument("--n", type=int, default=128, help="cells per side")
    ap.add_argument("--dx", type=float, default=PAPER_PARAMS["dx"],
                    help="grid spacing (with --n: the same domain at another resolution)")
    a = ap.parse_args(argv)
    r = run(a.t_end, a.precision, n=a.n, every=a.every, params=dict(dx=a.dx),
            log=lambda s: print(s, flush=True))
    summary = {k: v for k, v in r.items() if k != "rho"}
    print(json.dumps({k: v for k, v in summary.items() if k not in ("times", "e_T")}), flush=True)
    if a.json:
        json.dump(summary, open(a.json, "w"))
    if a.npz:
        np.savez(a.npz, **{f"rho_t{t:g}": v for t, v in r["rho"].items()})


if __name__ == "__main__":
    sys.exit(main())
