"""Pins of the oracle's force coefficients B, C, C_q (Eq. 2 and the NS system of Sec. 2.2) and of
its total-energy diagnostic e_T (Sec. 2.2) against exact calculus.

The fields are trigonometric polynomials of degree <= 2 per axis on a periodic square of side
2 pi, sampled on a 64-point grid.  There the windowed-FFT wavenumber of Eq. (3) equals the exact
wavenumber to round-off for the modes these fields and their smooth pointwise functions carry
(the truncated arcsin series is exact to ~1e-13 up to mode N/8, and the spectra of the rational
functions of these small-amplitude fields decay geometrically), so the oracle's spectral
derivatives reproduce the exact derivatives.  The grid is kept small because the round-off of
composed spectral derivatives grows with the highest wavenumber: B holds the divergence of
rho lap rho, a third derivative, whose round-off grows as N^3 (about 3e-12 of max|B| at N = 64,
1.4e-11 at N = 96).  The expected values are the paper's printed formulas differentiated exactly
by sympy, in their expanded (non-divergence) form, with grad(M/T) differentiated as written
(no chain-rule reading), and with T, u and rho all non-uniform, H != 0 and q != 0.

Negative controls: each plausible slip (a flipped sign of the thermal term of Lambda, T instead
of T^2 in C_q's denominator, rho dropped inside C_q's divergence, K instead of K/2 in e_T) moves
the expected values far outside the tolerance, so each would fail the pin.
"""
import functools

import numpy as np
import pytest
import sympy as sp

from oracle import dvm, model

N = 64
L = 2 * np.pi
H_DX = L / N

X, Y = sp.symbols("x y", real=True)

# Parameters with every term of B, C, C_q switched on (the paper's fluid would be a = 9/8,
# b_w = 1/3; the benchmark fluid is used here).
PAR = dict(K=sp.Rational(4, 1000), H=sp.Rational(3, 1000), zeta=sp.Rational(1, 100),
           q=sp.Rational(-2, 100), a=sp.Rational(9, 49), bw=sp.Rational(2, 21), b=2)


def _trig(rng, c0, amp, modes):
    """c0 + amp * sum over modes of r_k cos(kx x + ky y + phi_k), with rational r_k, phi_k."""
    e = sp.nsimplify(c0)
    for kx, ky in modes:
        r = sp.Rational(int(rng.integers(300, 1000)), 1000)
        ph = sp.Rational(int(rng.integers(0, 6283)), 1000)
        e = e + sp.nsimplify(amp) * r * sp.cos(kx * X + ky * Y + ph)
    return e


@functools.lru_cache(maxsize=None)
def _fields(seed):
    rng = np.random.default_rng(seed)
    rho = _trig(rng, 3, sp.Rational(6, 100), [(1, 0), (0, 1), (1, 2), (2, -1)])
    ux = _trig(rng, sp.Rational(1, 100), sp.Rational(2, 100), [(1, 1), (0, 2), (2, 0)])
    uy = _trig(rng, sp.Rational(-1, 100), sp.Rational(2, 100), [(1, 0), (1, -2), (0, 1)])
    T = _trig(rng, sp.Rational(1, 2), sp.Rational(15, 1000), [(0, 1), (2, 1), (1, -1)])
    return rho, ux, uy, T


def _grad(g):
    return sp.diff(g, X), sp.diff(g, Y)


def _div(vx, vy):
    return sp.diff(vx, X) + sp.diff(vy, Y)


def _exact_coefficients(rho, ux, uy, T, lam_sign=1, cq_power=2, cq_rho=True):
    """B_x, B_y, C, C_q as printed in Sec. 2.2, with exact derivatives.

    B = [grad(P^w - rho T) + div Lambda - grad(zeta div u)] / (rho T)
    C = {(P^w - rho T) div u + Lambda : grad u - zeta (div u)^2 + a rho^2 div u
         + K [-(grad rho . grad rho) div u / 2 - rho grad rho . grad(div u)
              - grad rho . grad u . grad rho]} / (2 rho T^2)
    C_q = div(q rho T grad T) / (rho T^2)
    Lambda = M grad rho grad rho - M (rho lap rho + |grad rho|^2/2) I
             - [rho T grad rho . grad(M/T)] I,   M = K + H T.
    The keyword arguments plant the slips of the negative controls."""
    K, Hc, zeta, q, a, bw = (PAR[k] for k in ("K", "H", "zeta", "q", "a", "bw"))
    rx, ry = _grad(rho)
    lap = sp.diff(rho, X, 2) + sp.diff(rho, Y, 2)
    Pw = rho * T / (1 - bw * rho) - a * rho ** 2
    M = K + Hc * T
    mtx, mty = _grad(M / T)
    iso = -M * (rho * lap + (rx ** 2 + ry ** 2) / 2) - lam_sign * rho * T * (rx * mtx + ry * mty)
    lam = [[M * rx * rx + iso, M * rx * ry], [M * ry * rx, M * ry * ry + iso]]
    div = _div(ux, uy)
    pn = Pw - rho * T
    # (div Lambda)_b = d_a Lambda_ab
    Bx = (sp.diff(pn, X) + sp.diff(lam[0][0], X) + sp.diff(lam[1][0], Y) - sp.diff(zeta * div, X)) / (rho * T)
    By = (sp.diff(pn, Y) + sp.diff(lam[0][1], X) + sp.diff(lam[1][1], Y) - sp.diff(zeta * div, Y)) / (rho * T)
    gu = [[sp.diff(ux, X), sp.diff(uy, X)], [sp.diff(ux, Y), sp.diff(uy, Y)]]   # (grad u)_ab = d_a u_b
    lam_du = sum(lam[i][j] * gu[i][j] for i in range(2) for j in range(2))
    gr = (rx, ry)
    rgr = sum(gr[i] * gu[i][j] * gr[j] for i in range(2) for j in range(2))
    gdx, gdy = _grad(div)
    num = (pn * div + lam_du - zeta * div ** 2 + a * rho ** 2 * div
           + K * (-(rx ** 2 + ry ** 2) * div / 2 - rho * (rx * gdx + ry * gdy) - rgr))
    C = num / (2 * rho * T ** 2)
    qr = rho if cq_rho else 1
    Cq = _div(q * qr * T * sp.diff(T, X), q * qr * T * sp.diff(T, Y)) / (rho * T ** cq_power)
    return Bx, By, C, Cq


def _grid():
    yy, xx = np.meshgrid(np.arange(N) * H_DX, np.arange(N) * H_DX, indexing="ij")
    return xx, yy


def _on_grid(expr):
    xx, yy = _grid()
    f = sp.lambdify((X, Y), expr, modules="numpy", cse=True)
    return np.broadcast_to(np.asarray(f(xx, yy), dtype=np.float64), xx.shape)


def _params(b=2):
    p = {k: float(v) for k, v in PAR.items()}
    p.update(dx=H_DX, dt=1e-3, tau=1e-2, b=float(b))
    return p


@functools.lru_cache(maxsize=None)
def _oracle(seed):
    fields = [_on_grid(e) for e in _fields(seed)]
    return fields, model.force_coefficients(*fields, _params())


@functools.lru_cache(maxsize=None)
def _expected(seed, **slip):
    return [_on_grid(e) for e in _exact_coefficients(*_fields(seed), **slip)]


def _rel(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


@pytest.mark.parametrize("seed", [11, 12])
def test_force_coefficients_match_exact_calculus(seed):
    (rho, ux, uy, T), got = _oracle(seed)
    # the state really exercises every term: non-uniform T, u and rho
    for g in (ux, uy, T):
        assert np.ptp(g) > 1e-3
    want = _expected(seed)
    for name, g, w in zip(("Bx", "By", "C", "Cq"), got, want):
        assert _rel(g, w) < 1e-11, (name, _rel(g, w))


def test_thermal_lambda_term_sign_is_pinned():
    # -rho T (grad rho . grad(M/T)) I with its sign flipped changes B and C far beyond the tolerance
    _, got = _oracle(11)
    bad = _expected(11, lam_sign=-1)
    assert _rel(got[0], bad[0]) > 1e-5 and _rel(got[1], bad[1]) > 1e-5
    assert _rel(got[2], bad[2]) > 1e-5


def test_thermal_lambda_term_is_the_full_gradient_of_m_over_t():
    # dropping the thermal term (as a uniform-T reading would) fails too
    _, got = _oracle(11)
    bad = _expected(11, lam_sign=0)
    assert _rel(got[0], bad[0]) > 1e-5 and _rel(got[2], bad[2]) > 1e-5


@pytest.mark.parametrize("slip", [dict(cq_power=1), dict(cq_rho=False)])
def test_cq_form_is_pinned(slip):
    # T^1 instead of T^2 in the denominator, or rho dropped inside the divergence, fails
    _, got = _oracle(11)
    bad = _expected(11, **slip)
    assert _rel(got[3], bad[3]) > 1e-3


def test_cq_energy_source_sums_to_zero():
    # 2 rho T^2 C_q = 2 div(q rho T grad T): the heat-conduction source of the energy moment of
    # I_i is a divergence, so its grid sum vanishes (a wrong power of T would not)
    (rho, ux, uy, T), (_, _, _, Cq) = _oracle(12)
    s = rho * T * T * Cq
    assert abs(s.sum()) < 1e-12 * np.abs(s).sum()
    assert abs((rho * T * Cq).sum()) > 1e-4 * np.abs(rho * T * Cq).sum()


# ---------------------------------------------------------------------------------------------
# Total energy e_T = rho T - a rho^2 + K |grad rho|^2/2 + rho u^2/2 (Sec. 2.2, b = 2); with b
# degrees of freedom the kinetic part is sum f (v^2 + eta^2)/2 = rho (b T + u^2)/2.

def _exact_energy_density(rho, ux, uy, T, b, k_half=True):
    K, a = PAR["K"], PAR["a"]
    rx, ry = _grad(rho)
    kc = K / 2 if k_half else K
    return rho * (b * T + ux ** 2 + uy ** 2) / 2 - a * rho ** 2 + kc * (rx ** 2 + ry ** 2)


@pytest.mark.parametrize("b", [2, 3])
def test_total_energy_density_matches_closed_form(b):
    rho_e, ux_e, uy_e, T_e = _fields(13)
    fields = [_on_grid(e) for e in (rho_e, ux_e, uy_e, T_e)]
    p = _params(b=b)
    f = model.init_equilibrium(*fields, p)
    got = model.total_energy_density(f, p)
    want = _on_grid(_exact_energy_density(rho_e, ux_e, uy_e, T_e, b))
    assert _rel(got, want) < 1e-12
    if b == 2:
        # the printed form rho T - a rho^2 + K |grad rho|^2/2 + rho u^2/2, term by term
        printed = _on_grid(rho_e * T_e - PAR["a"] * rho_e ** 2
                           + PAR["K"] * (sp.diff(rho_e, X) ** 2 + sp.diff(rho_e, Y) ** 2) / 2
                           + rho_e * (ux_e ** 2 + uy_e ** 2) / 2)
        assert _rel(got, printed) < 1e-12
    bad = _on_grid(_exact_energy_density(rho_e, ux_e, uy_e, T_e, b, k_half=False))
    assert np.abs(got - bad).max() > 1e-4 * np.abs(want).max() * 1e-2


def test_total_energy_integral_matches_exact_integral():
    # The grid integral of e_T (conservation()[3]) against sympy's exact integral over the
    # periodic square, for a state small enough to integrate symbolically: every term of e_T
    # (the kinetic, van der Waals and gradient parts) contributes at a different order.
    rho_e = 3 + sp.Rational(1, 10) * sp.cos(X + sp.Rational(1, 3)) + sp.Rational(1, 20) * sp.sin(2 * Y)
    ux_e = sp.Rational(3, 100) * sp.sin(Y)
    uy_e = sp.Rational(1, 50) * sp.cos(X - Y)
    T_e = sp.Rational(1, 2) + sp.Rational(1, 50) * sp.cos(X)
    b = 2
    dens = _exact_energy_density(rho_e, ux_e, uy_e, T_e, b)
    exact = float(sp.integrate(sp.integrate(sp.expand(dens), (X, 0, 2 * sp.pi)), (Y, 0, 2 * sp.pi)))
    fields = [_on_grid(e) for e in (rho_e, ux_e, uy_e, T_e)]
    p = _params(b=b)
    f = model.init_equilibrium(*fields, p)
    got = model.conservation(f, p)[3]
    assert abs(got - exact) < 1e-12 * abs(exact)
    # the gradient part alone is ~2e-4 of the total: a K (instead of K/2) slip is visible
    grad_part = float(sp.integrate(sp.integrate(sp.expand(PAR["K"] / 2 * (sp.diff(rho_e, X) ** 2 + sp.diff(rho_e, Y) ** 2)),
                                                (X, 0, 2 * sp.pi)), (Y, 0, 2 * sp.pi)))
    assert abs(grad_part) > 1e3 * 1e-12 * abs(exact)


def test_equilibrium_energy_moment_is_rho_b_t_plus_u2():
    # the energy moment of f^eq the e_T diagnostic starts from (Sec. 2.1 with the rho reading)
    rng = np.random.default_rng(3)
    rho, ux, uy, T = rng.uniform(2, 4, 7), rng.uniform(-.1, .1, 7), rng.uniform(-.1, .1, 7), rng.uniform(.4, .6, 7)
    for b in (2.0, 3.0):
        f = dvm.equilibrium(rho, ux, uy, T, b)
        vx, vy, eta = dvm.velocities()
        e = np.tensordot(vx * vx + vy * vy + eta * eta, f, axes=(0, 0))
        assert np.abs(e - rho * (b * T + ux * ux + uy * uy)).max() < 1e-13 * e.max()
