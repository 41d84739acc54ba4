"""Shared helpers of the GPU parity tests (no method arithmetic here)."""
import sys

import numpy as np


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel(a, b):
    """max |a - b| / max |b|."""
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def field_errors(f_gpu, f_ref, moments):
    """Parity norm: rho and T relative to their max, u relative to sqrt(max T), f relative to
    max |f|."""
    r1, ux1, uy1, T1 = moments(f_gpu)
    r0, ux0, uy0, T0 = moments(f_ref)
    s = np.sqrt(np.abs(T0).max())
    return dict(rho=rel(r1, r0), T=rel(T1, T0),
                u=float(max(np.abs(ux1 - ux0).max(), np.abs(uy1 - uy0).max()) / s),
                f=rel(f_gpu, f_ref))
