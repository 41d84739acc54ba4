"""Moments, forcing term, right-hand side of Eq. (1) and the two-stage Runge-Kutta step.
Test infrastructure only.

Parameters are a plain dict ``p`` with keys dx, dt, tau, K, H, zeta, q, b, a, bw and an
optional ``dvm`` dict (ring speeds and eta0, see ``oracle.dvm``).  Fields are float64 arrays
[ny, nx] (populations [16, ny, nx]), row-major with x the fast axis.

Readings of points the paper leaves open (each also listed in the design notes):
* moments: the energy moment is rho (b T + u^2) = sum f (v^2 + eta^2) (the printed form omits
  rho on the left);
* the hard-coded 9/8 of the paper's C and e_T is the EOS parameter a;
* nabla(M/T) with M = K + H T and H constant is the chain rule -K nabla T / T^2;
* nabla.Lambda and the other divergences of B are taken in divergence form of the stress
  S = (P^w - rho T) I + Lambda - zeta (div u) I;
* the printed "- zeta (div u)" inside C is read as the dissipation - zeta (div u)^2;
* the RK2 stage update has the signs of Eq. (1): f^{n+1/2} = f^n + dt/2 R(f^n),
  f^{n+1} = f^n + dt R(f^{n+1/2}) with R = -v.grad f - (f - f^eq)/tau + I.
"""
import numpy as np

from . import dvm as _dvm
from .spectral import dx_, dy_


def moments(f, p):
    """rho, ux, uy, T of populations f[16, ...] (Sec. 2.1)."""
    vx, vy, eta = _dvm.velocities(p.get("dvm"))
    sh = (16,) + (1,) * (f.ndim - 1)
    rho = f.sum(axis=0)
    ux = (f * vx.reshape(sh)).sum(axis=0) / rho
    uy = (f * vy.reshape(sh)).sum(axis=0) / rho
    e2 = (f * (vx * vx + vy * vy + eta * eta).reshape(sh)).sum(axis=0)
    T = (e2 / rho - ux * ux - uy * uy) / p["b"]
    return rho, ux, uy, T


def force_coefficients(rho, ux, uy, T, p):
    """B_x, B_y, C, C_q of Eq. (2) from the macroscopic fields (Sec. 2.2).

    P^w = rho T/(1 - b_w rho) - a rho^2;  M = K + H T;
    Lambda = M grad rho grad rho - M (rho lap rho + |grad rho|^2/2) I - rho T (grad rho . grad(M/T)) I;
    B = div S / (rho T) with S = (P^w - rho T) I + Lambda - zeta (div u) I;
    C = [(P^w - rho T) div u + Lambda : grad u - zeta (div u)^2 + a rho^2 div u
         + K (-|grad rho|^2 div u / 2 - rho grad rho . grad(div u) - d_a rho d_a u_b d_b rho)]
        / (2 rho T^2);
    C_q = div(q rho T grad T) / (rho T^2).
    """
    h = p["dx"]
    K, H, zeta, q, a, bw = p["K"], p["H"], p["zeta"], p["q"], p["a"], p["bw"]

    rx, ry = dx_(rho, h), dy_(rho, h)
    lap = dx_(rx, h) + dy_(ry, h)
    Tx, Ty = dx_(T, h), dy_(T, h)
    uxx, uxy = dx_(ux, h), dy_(ux, h)      # d_x u_x, d_y u_x
    uyx, uyy = dx_(uy, h), dy_(uy, h)      # d_x u_y, d_y u_y
    div = uxx + uyy
    gdx, gdy = dx_(div, h), dy_(div, h)

    Pw = rho * T / (1.0 - bw * rho) - a * rho * rho
    M = K + H * T
    g2 = rx * rx + ry * ry
    # grad(M/T) = -K grad T / T^2 for constant H
    mtx, mty = -K * Tx / (T * T), -K * Ty / (T * T)
    iso = -M * (rho * lap + 0.5 * g2) - rho * T * (rx * mtx + ry * mty)
    Lxx = M * rx * rx + iso
    Lxy = M * rx * ry
    Lyy = M * ry * ry + iso

    Sxx = Pw - rho * T + Lxx - zeta * div
    Sxy = Lxy
    Syy = Pw - rho * T + Lyy - zeta * div
    Bx = (dx_(Sxx, h) + dy_(Sxy, h)) / (rho * T)
    By = (dx_(Sxy, h) + dy_(Syy, h)) / (rho * T)

    # Lambda : grad u with (grad u)_{ab} = d_a u_b
    lam_du = Lxx * uxx + Lxy * uyx + Lxy * uxy + Lyy * uyy
    # d_a rho (d_a u_b) d_b rho
    rgr = rx * (uxx * rx + uyx * ry) + ry * (uxy * rx + uyy * ry)
    num = ((Pw - rho * T) * div + lam_du - zeta * div * div + a * rho * rho * div
           + K * (-0.5 * g2 * div - rho * (rx * gdx + ry * gdy) - rgr))
    C = num / (2.0 * rho * T * T)

    Cq = (dx_(q * rho * T * Tx, h) + dy_(q * rho * T * Ty, h)) / (rho * T * T)
    return Bx, By, C, Cq


def forcing(feq, rho, ux, uy, T, Bx, By, C, Cq, p):
    """I_i of Eq. (2): -[A + B.(v_i - u) + (C + C_q)|v_i - u|^2] f_i^eq, A = -2 (C + C_q) T."""
    vx, vy, _ = _dvm.velocities(p.get("dvm"))
    sh = (16,) + (1,) * rho.ndim
    cx = vx.reshape(sh) - ux
    cy = vy.reshape(sh) - uy
    D = C + Cq
    A = -2.0 * D * T
    return -(A + Bx * cx + By * cy + D * (cx * cx + cy * cy)) * feq


def rhs(f, p):
    """R(f) = -v_i . grad f_i - (f_i - f_i^eq)/tau + I_i (Eq. 1)."""
    vx, vy, _ = _dvm.velocities(p.get("dvm"))
    sh = (16,) + (1,) * (f.ndim - 1)
    rho, ux, uy, T = moments(f, p)
    feq = _dvm.equilibrium(rho, ux, uy, T, p["b"], p.get("dvm"))
    Bx, By, C, Cq = force_coefficients(rho, ux, uy, T, p)
    I = forcing(feq, rho, ux, uy, T, Bx, By, C, Cq, p)
    adv = vx.reshape(sh) * dx_(f, p["dx"]) + vy.reshape(sh) * dy_(f, p["dx"])
    return -adv - (f - feq) / p["tau"] + I


def rk2_step(f, p):
    """One step of the two-stage (midpoint) Runge-Kutta scheme of Sec. 2.3."""
    dt = p["dt"]
    f_half = f + 0.5 * dt * rhs(f, p)
    return f + dt * rhs(f_half, p)


def run(f, p, n):
    for _ in range(n):
        f = rk2_step(f, p)
    return f


def init_equilibrium(rho, ux, uy, T, p):
    """Initial populations f = f^eq(rho0, u0, T0) (the paper does not state its start)."""
    return _dvm.equilibrium(rho, ux, uy, T, p["b"], p.get("dvm"))


def total_energy_density(f, p):
    """e_T = sum f (v^2 + eta^2)/2 - a rho^2 + K |grad rho|^2/2 (Sec. 2.2; at b = 2 this is the
    printed rho T - a rho^2 + K |grad rho|^2/2 + rho u^2/2)."""
    vx, vy, eta = _dvm.velocities(p.get("dvm"))
    sh = (16,) + (1,) * (f.ndim - 1)
    rho = f.sum(axis=0)
    kin = 0.5 * (f * (vx * vx + vy * vy + eta * eta).reshape(sh)).sum(axis=0)
    rx, ry = dx_(rho, p["dx"]), dy_(rho, p["dx"])
    return kin - p["a"] * rho * rho + 0.5 * p["K"] * (rx * rx + ry * ry)


def conservation(f, p):
    """Grid sums (times cell area) of mass, x- and y-momentum and total energy."""
    vx, vy, _ = _dvm.velocities(p.get("dvm"))
    area = p["dx"] * p["dx"]
    sh = (16,) + (1,) * (f.ndim - 1)
    mass = f.sum() * area
    mx = (f * vx.reshape(sh)).sum() * area
    my = (f * vy.reshape(sh)).sum() * area
    e = total_energy_density(f, p).sum() * area
    return np.array([mass, mx, my, e])
