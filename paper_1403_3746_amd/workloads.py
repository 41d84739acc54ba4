"""Seeded synthetic workloads: parameter sets and initial (rho, u, T) fields.

This module holds no arithmetic of the lattice Boltzmann method itself -- only the recipes
that build inputs.  The same arrays feed the HIP library and, in the tests, the CPU oracle.

The paper's runs use analytic initial conditions (a flat liquid slab, Sec. 3.1; a quench with
small random density noise, Sec. 3.2), so synthetic inputs of those shapes are the real
workloads.  The benchmark family uses a van der Waals fluid with a = 9/49, b_w = 2/21 (critical
point T_c = 4/7, rho_c = 7/2), dx = 1, dt = 1e-3, tau = 1e-2, K = 1e-2, b = 2, H = zeta = q = 0.
"""
import numpy as np

T_C = 4.0 / 7.0
RHO_C = 3.5
VDW_A = 9.0 / 49.0
VDW_BW = 2.0 / 21.0

# Line lengths of the ragged batch (the library takes 2^a or 3*2^a from 8 to 2048).
RAGGED_SIZES = (64, 96, 128, 192, 256, 384, 512, 1024)


def base_params(**over):
    p = dict(dx=1.0, dt=1e-3, tau=1e-2, K=1e-2, H=0.0, zeta=0.0, q=0.0, b=2.0,
             a=VDW_A, bw=VDW_BW)
    p.update(over)
    return p


def slab(nx, ny, T):
    """Flat liquid slab: rho(x_j) = rho_c + 1.5 tanh((nx/4 - |j - nx/2|)/2), uniform in y;
    liquid in the middle half as in the coexistence runs of Sec. 3.1."""
    j = np.arange(nx, dtype=np.float64)
    prof = RHO_C + 1.5 * np.tanh((nx / 4.0 - np.abs(j - nx / 2.0)) / 2.0)
    rho = np.broadcast_to(prof[None, :], (ny, nx)).copy()
    z = np.zeros((ny, nx))
    return rho, z.copy(), z.copy(), np.full((ny, nx), float(T))


def quench(nx, ny, T, seed, amp=1e-3):
    """Thermal quench: rho = rho_c (1 + amp U(-1,1)) i.i.d. per cell, u = 0, uniform T (Sec. 3.2)."""
    rng = np.random.default_rng(seed)
    rho = RHO_C * (1.0 + amp * rng.uniform(-1.0, 1.0, (ny, nx)))
    z = np.zeros((ny, nx))
    return rho, z.copy(), z.copy(), np.full((ny, nx), float(T))


def smooth_random(nx, ny, seed, T0=0.5, rho0=RHO_C, drho=0.3, du=0.05, dT=0.03, modes=3):
    """A band-limited random state with non-zero velocity and temperature gradients, for unit
    parity tests of every term (the benchmark states start at rest with uniform T)."""
    rng = np.random.default_rng(seed)
    y, x = np.meshgrid(np.arange(ny) / ny, np.arange(nx) / nx, indexing="ij")

    def field(amp):
        g = np.zeros((ny, nx))
        for kx in range(-modes, modes + 1):
            for ky in range(-modes, modes + 1):
                if kx == 0 and ky == 0:
                    continue
                c, ph = rng.normal() / (1 + kx * kx + ky * ky), rng.uniform(0, 2 * np.pi)
                g += c * np.cos(2 * np.pi * (kx * x + ky * y) + ph)
        return amp * g / max(np.abs(g).max(), 1e-30)

    return rho0 + field(drho), field(du), field(du), T0 + field(dT)


def config(name):
    """Named benchmark workloads: list of (params, (rho, ux, uy, T)) per instance, plus steps."""
    if name == "slab64":
        p = base_params()
        return [(p, slab(64, 64, 0.9 * T_C))], 100
    if name == "quench512":
        p = base_params()
        return [(p, quench(512, 512, 0.9 * T_C, 2000))], 10000
    if name == "quench2048":
        # FP32 state with the FP64 mass/energy reductions run every step (a history ring)
        p = base_params(hist=5000)
        return [(p, quench(2048, 2048, 0.85 * T_C, 3000))], 5000
    if name == "batch128x256":
        Ts = T_C * (0.85 + 0.13 * np.random.default_rng(4999).uniform(size=256))
        return [(base_params(), quench(128, 128, Ts[k], 4000 + k)) for k in range(256)], 2000
    if name == "ragged64":
        rng = np.random.default_rng(5999)
        ns = rng.choice(RAGGED_SIZES, size=64)
        Ts = T_C * (0.85 + 0.13 * rng.uniform(size=64))
        out = []
        for k in range(64):
            n = int(ns[k])
            ic = slab(n, n, Ts[k]) if k % 2 == 0 else quench(n, n, Ts[k], 5000 + k)
            out.append((base_params(), ic))
        return out, 1000
    raise KeyError(name)
