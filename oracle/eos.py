"""Van der Waals equation of state and Maxwell construction.  Test infrastructure only.

The paper prints P^w = 3 rho T/(3 - rho) - (9/8) rho^2 (Sec. 2.2, NS system), i.e. the general
form P^w = rho T/(1 - b_w rho) - a rho^2 with a = 9/8, b_w = 1/3 (T_c = rho_c = 1).  Coexistence
densities (Sec. 3.1 compares the model's curve with them; Sec. 3.3 uses the pair at T = 0.95)
follow from equal pressure and equal chemical potential.
"""
import numpy as np
from scipy.optimize import brentq


def pressure(rho, T, a, bw):
    return rho * T / (1.0 - bw * rho) - a * rho * rho


def chemical_potential(rho, T, a, bw):
    """mu(rho) up to a T-dependent constant; d mu/d rho = (1/rho) dP/d rho at fixed T."""
    return (T * np.log(rho / (1.0 - bw * rho)) + T * bw * rho / (1.0 - bw * rho)
            - 2.0 * a * rho)


def critical_point(a, bw):
    """(T_c, rho_c, P_c) of the van der Waals fluid."""
    return 8.0 * a / (27.0 * bw), 1.0 / (3.0 * bw), a / (27.0 * bw * bw)


def spinodals(T, a, bw):
    """Densities where dP/d rho = 0 (below T_c): vapour spinodal < rho_c < liquid spinodal."""
    _, rc, _ = critical_point(a, bw)
    dp = lambda r: T / (1.0 - bw * r) ** 2 - 2.0 * a * r
    lo = brentq(dp, 1e-9, rc)
    hi = brentq(dp, rc, (1.0 - 1e-12) / bw)
    return lo, hi


def maxwell(T, a, bw):
    """Coexisting (rho_vapour, rho_liquid) at temperature T < T_c.

    For a trial saturation pressure P between the two spinodal pressures, the vapour and
    liquid branches give rho_v(P) < spinodal_lo and rho_l(P) > spinodal_hi; the coexistence
    pressure is the root of mu(rho_v(P)) - mu(rho_l(P))."""
    s_lo, s_hi = spinodals(T, a, bw)
    p_lo, p_hi = pressure(s_hi, T, a, bw), pressure(s_lo, T, a, bw)
    rmax = (1.0 - 1e-13) / bw

    def branches(P):
        rv = brentq(lambda r: pressure(r, T, a, bw) - P, 1e-14, s_lo, xtol=1e-15, rtol=1e-15)
        rl = brentq(lambda r: pressure(r, T, a, bw) - P, s_hi, rmax, xtol=1e-15, rtol=1e-15)
        return rv, rl

    def dmu(P):
        rv, rl = branches(P)
        return chemical_potential(rv, T, a, bw) - chemical_potential(rl, T, a, bw)

    eps = 1e-12 * max(abs(p_hi - p_lo), 1e-300)
    Psat = brentq(dmu, max(p_lo, 0.0) + eps, p_hi - eps, xtol=1e-15, rtol=1e-15)
    rv, rl = branches(Psat)
    return float(rv), float(rl)
