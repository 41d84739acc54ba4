"""Pins of the windowed-FFT derivative (Sec. 2.3, Eq. 3) against mathematics, not itself."""
import math
import os

import numpy as np
import pytest

from oracle import spectral

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_series_coefficients_are_arcsin_taylor():
    # Printed coefficients (golden file) equal the arcsin Maclaurin coefficients
    # C(2n, n) / (4^n (2n + 1)), and the oracle uses exactly these.
    rows = [l.split() for l in open(os.path.join(GOLDEN, "arcsin_series_eq3.txt"))
            if l.strip() and not l.startswith("#")]
    printed = [int(a) / int(b) for a, b in rows]
    taylor = [math.comb(2 * n, n) / (4 ** n * (2 * n + 1)) for n in range(8)]
    assert np.allclose(printed, taylor, rtol=0, atol=1e-17)
    assert np.allclose(spectral.ARCSIN_SERIES, taylor, rtol=0, atol=1e-17)


def test_series_within_truncation_bound_of_arcsin():
    # |arcsin(phi) - S(phi)| <= c_8 phi^17 / (1 - phi^2), c_8 the first dropped coefficient.
    c8 = math.comb(16, 8) / (4 ** 8 * 17)
    phi = np.linspace(0.0, 0.95, 400)
    err = np.abs(np.arcsin(phi) - spectral.series(phi))
    bound = c8 * phi ** 17 / (1 - phi ** 2) + 1e-15
    assert np.all(err <= bound)
    # at phi = 1 the truncated series is 0.8724 of pi/2
    assert abs(spectral.series(1.0) / (np.pi / 2) - 0.87241) < 1e-5


@pytest.mark.parametrize("n", [8, 12, 64, 96])
def test_wavenumber_relative_error(n):
    dx = 0.37
    k = spectral.wavenumber(n, dx)
    m = np.arange(n)
    ms = np.where(m < (n + 1) // 2, m, m - n)
    exact = 2 * np.pi * ms / (n * dx)
    # odd symmetry and zero DC / Nyquist
    assert k[0] == 0.0
    if n % 2 == 0:
        assert k[n // 2] == 0.0
    assert np.allclose(k[1:], -k[1:][::-1], rtol=0, atol=1e-14)
    if n >= 64:
        for frac, tol in ((8, 3e-9), (4, 8e-5), (1e9, 1e-15)):
            mm = max(1, int(n // frac)) if frac < 1e9 else 1
            rel = abs(k[mm] - exact[mm]) / exact[mm]
            assert rel < tol, (mm, rel)


def _naive_dft_derivative(g, dx, axis):
    """Brute-force O(N^2) DFT derivative along one axis of a 2-D field."""
    g = np.moveaxis(g, axis, -1)
    n = g.shape[-1]
    k = spectral.wavenumber(n, dx)
    out = np.zeros_like(g)
    for r in range(g.shape[0]):
        for j in range(n):
            acc = 0.0 + 0.0j
            for m in range(n):
                gm = sum(g[r, l] * complex(math.cos(2 * math.pi * m * l / n),
                                           -math.sin(2 * math.pi * m * l / n)) for l in range(n))
                acc += 1j * k[m] * gm * complex(math.cos(2 * math.pi * m * j / n),
                                                math.sin(2 * math.pi * m * j / n))
            out[r, j] = (acc / n).real
    return np.moveaxis(out, -1, axis)


def test_derivative_matches_naive_dft_8x8():
    rng = np.random.default_rng(11)
    g = rng.normal(size=(8, 8))
    dx = 0.8
    assert np.allclose(spectral.dx_(g, dx), _naive_dft_derivative(g, dx, axis=1), rtol=0, atol=1e-12)
    assert np.allclose(spectral.dy_(g, dx), _naive_dft_derivative(g, dx, axis=0), rtol=0, atol=1e-12)
    # rectangular grid, 6 x 8
    g2 = rng.normal(size=(6, 8))
    assert np.allclose(spectral.dx_(g2, dx), _naive_dft_derivative(g2, dx, axis=1), atol=1e-12)
    assert np.allclose(spectral.dy_(g2, dx), _naive_dft_derivative(g2, dx, axis=0), atol=1e-12)


def test_derivative_of_band_limited_fields_is_exact():
    ny, nx, dx = 48, 64, 0.25
    y, x = np.meshgrid(np.arange(ny) * dx, np.arange(nx) * dx, indexing="ij")
    Lx, Ly = nx * dx, ny * dx
    ax, ay = 2 * np.pi * 3 / Lx, 2 * np.pi * 2 / Ly
    g = np.sin(ax * x + 0.3) * np.cos(ay * y) + 0.5 * np.cos(2 * np.pi * x / Lx)
    gx = ax * np.cos(ax * x + 0.3) * np.cos(ay * y) - 0.5 * (2 * np.pi / Lx) * np.sin(2 * np.pi * x / Lx)
    gy = -ay * np.sin(ax * x + 0.3) * np.sin(ay * y)
    assert np.abs(spectral.dx_(g, dx) - gx).max() < 1e-13
    assert np.abs(spectral.dy_(g, dx) - gy).max() < 1e-13
    # second derivative as a composition
    gxx = -ax * ax * np.sin(ax * x + 0.3) * np.cos(ay * y) - 0.5 * (2 * np.pi / Lx) ** 2 * np.cos(2 * np.pi * x / Lx)
    assert np.abs(spectral.dx_(spectral.dx_(g, dx), dx) - gxx).max() < 1e-12


def test_high_mode_uses_truncated_series():
    # at m = N/4 the derivative is attenuated exactly by S(phi)/arcsin(phi)
    n, dx = 64, 1.0
    x = np.arange(n) * dx
    g = np.broadcast_to(np.sin(2 * np.pi * 16 * x / n), (4, n))
    d = spectral.dx_(g, dx)
    phi = np.sin(np.pi * 16 / n)
    kappa = (2 / dx) * sum(math.comb(2 * j, j) / (4 ** j * (2 * j + 1)) * phi ** (2 * j + 1) for j in range(8))
    assert np.abs(d - kappa * np.cos(2 * np.pi * 16 * x / n)).max() < 1e-13
    assert abs(kappa / (2 * np.pi * 16 / n) - 1) > 1e-5      # visibly not the exact wavenumber


def test_nyquist_and_mean():
    n = 16
    g = np.broadcast_to(((-1.0) ** np.arange(n)), (n, n)).copy()
    assert np.abs(spectral.dx_(g, 1.0)).max() < 1e-14
    assert np.abs(spectral.dy_(g.T, 1.0)).max() < 1e-14
    rng = np.random.default_rng(3)
    r = rng.normal(size=(n, n))
    assert abs(spectral.dx_(r, 0.5).sum()) < 1e-12
    assert abs(spectral.dy_(r, 0.5).sum()) < 1e-12
