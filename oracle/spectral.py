"""Windowed-FFT spectral derivative (Sec. 2.3, Eq. 3).  Test infrastructure only.

For an axis of length N and spacing dx, mode m has signed index m' (m' = m for m < N/2, else
m - N), phi = sin(pi m'/N) = sin(k dx / 2) and the multiplier k_x of Eq. (3): the arcsin series
truncated after the phi^15 term, times 2/dx.  For even N the Nyquist mode gets multiplier 0
(the paper is silent; 0 is the only value that keeps the derivative of a real field real).

D_x g = IFFT2[ i k_x(m_x) FFT2 g ] and likewise D_y.  Higher derivatives are compositions.
"""
import numpy as np
import scipy.fft as sfft

# Coefficients of phi, phi^3, ..., phi^15 printed in Eq. (3).
ARCSIN_SERIES = (1.0, 1.0 / 6.0, 3.0 / 40.0, 5.0 / 112.0, 35.0 / 1152.0,
                 63.0 / 2816.0, 231.0 / 13312.0, 143.0 / 10240.0)

_WORKERS = 1


def set_workers(n):
    """Threads scipy.fft may use (the CPU-baseline timing sets this; default 1)."""
    global _WORKERS
    _WORKERS = int(n)


def series(phi):
    """Truncated arcsin series of Eq. (3), evaluated term by term."""
    phi = np.asarray(phi, dtype=np.float64)
    s = np.zeros_like(phi)
    for j, c in enumerate(ARCSIN_SERIES):
        s = s + c * phi ** (2 * j + 1)
    return s


def wavenumber(n, dx):
    """k(m) of Eq. (3) for m = 0..n-1 (numpy FFT ordering)."""
    m = np.arange(n)
    msigned = np.where(m < (n + 1) // 2, m, m - n).astype(np.float64)
    phi = np.sin(np.pi * msigned / n)
    k = (2.0 / dx) * series(phi)
    if n % 2 == 0:
        k[n // 2] = 0.0
    return k


def dx_(g, dx):
    """D_x of real field(s) g[..., ny, nx] (x is the last axis)."""
    g = np.asarray(g, dtype=np.float64)
    ny, nx = g.shape[-2:]
    kx = wavenumber(nx, dx)[: nx // 2 + 1]
    G = sfft.rfft2(g, axes=(-2, -1), workers=_WORKERS)
    return sfft.irfft2(1j * kx[None, :] * G, s=(ny, nx), axes=(-2, -1), workers=_WORKERS)


def dy_(g, dx):
    """D_y of real field(s) g[..., ny, nx] (y is the second-last axis)."""
    g = np.asarray(g, dtype=np.float64)
    ny, nx = g.shape[-2:]
    ky = wavenumber(ny, dx)
    G = sfft.rfft2(g, axes=(-2, -1), workers=_WORKERS)
    return sfft.irfft2(1j * ky[:, None] * G, s=(ny, nx), axes=(-2, -1), workers=_WORKERS)
