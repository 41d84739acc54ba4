"""Pins of the D2V16 equilibrium (Sec. 2.1; seven kinetic moments, Sec. 2.2)."""
import numpy as np
import pytest

from oracle import dvm, model

# The 16 moment weights as monomials vx^p vy^q (v^2 + eta^2)^r (the seven kinetic moments).
PQR = [(0, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1), (2, 0, 0), (1, 1, 0), (0, 2, 0),
       (1, 0, 1), (0, 1, 1), (3, 0, 0), (2, 1, 0), (1, 2, 0), (0, 3, 0),
       (2, 0, 1), (1, 1, 1), (0, 2, 1)]


def continuous_maxwellian_moment(rho, ux, uy, T, b, p, q, r, order=12):
    """Gauss-Hermite quadrature of a Maxwellian in (vx, vy) plus b-2 internal degrees of
    freedom zeta (energy zeta^2 in place of eta^2): int f vx^p vy^q (v^2 + zeta^2)^r."""
    x, w = np.polynomial.hermite_e.hermegauss(order)
    s = np.sqrt(T)
    extra = int(round(b - 2))
    total = 0.0
    if extra == 0:
        zeta2 = [(0.0, 1.0)]
    else:
        # one extra degree of freedom: zeta ~ N(0, T)
        assert extra == 1
        zeta2 = [((s * xz) ** 2, wz / np.sqrt(2 * np.pi)) for xz, wz in zip(x, w)]
    for i, xi in enumerate(x):
        for j, xj in enumerate(x):
            vx, vy = ux + s * xi, uy + s * xj
            for z2, wz in zeta2:
                total += w[i] * w[j] * wz * vx ** p * vy ** q * (vx * vx + vy * vy + z2) ** r
    return rho * total / (2 * np.pi)


def test_moment_matrix_invertible_and_conditioned():
    vx, vy, eta = dvm.velocities()
    C = dvm.moment_matrix(vx, vy, eta)
    assert np.linalg.matrix_rank(C) == 16
    assert np.linalg.cond(C) < 200
    # without eta the (v^2 + eta^2) rows collapse onto the v^2 rows: rank 13
    assert np.linalg.matrix_rank(dvm.moment_matrix(vx, vy, 0 * eta)) == 13


@pytest.mark.parametrize("b", [2.0, 3.0])
@pytest.mark.parametrize("state", [(1.3, 0.0, 0.0, 0.5), (3.5, 0.12, -0.07, 0.514),
                                   (0.7, -0.2, 0.15, 0.45)])
def test_equilibrium_reproduces_continuous_maxwellian_moments(state, b):
    rho, ux, uy, T = state
    vx, vy, eta = dvm.velocities()
    feq = dvm.equilibrium(rho, ux, uy, T, b)
    for p, q, r in PQR:
        disc = float(np.sum(feq * vx ** p * vy ** q * (vx * vx + vy * vy + eta * eta) ** r))
        cont = continuous_maxwellian_moment(rho, ux, uy, T, b, p, q, r)
        assert abs(disc - cont) <= 1e-12 * max(1.0, abs(cont)), (p, q, r, disc, cont)


def test_moments_of_equilibrium_return_state():
    p = dict(b=2.0)
    rng = np.random.default_rng(5)
    rho = rng.uniform(0.5, 5, (6, 7))
    ux, uy = rng.uniform(-0.2, 0.2, (2, 6, 7))
    T = rng.uniform(0.4, 0.6, (6, 7))
    f = dvm.equilibrium(rho, ux, uy, T, 2.0)
    r2, ux2, uy2, T2 = model.moments(f, p)
    for a, b_ in ((rho, r2), (ux, ux2), (uy, uy2), (T, T2)):
        assert np.abs(a - b_).max() < 1e-13


def test_ring1_sums_to_zero_at_b2():
    # at b = 2 the M2,0 condition equals the trace of M2, so sum_i eta_i^2 f_i = 0
    f = dvm.equilibrium(2.0, 0.1, -0.05, 0.55, 2.0)
    assert abs(f[:4].sum()) < 1e-15 * 2.0 * 16


def _rot_perm():
    # member k of each ring -> member k+1 (rotation by +90 degrees)
    return np.array([(r * 4 + (k + 1) % 4) for r in range(4) for k in range(4)])


def test_rotation_and_mirror_permute_equilibrium():
    rho, ux, uy, T = 2.7, 0.13, -0.04, 0.49
    f = dvm.equilibrium(rho, ux, uy, T, 2.0)
    fr = dvm.equilibrium(rho, -uy, ux, T, 2.0)          # u rotated by +90 degrees
    perm = _rot_perm()
    assert np.abs(fr[perm] - f).max() < 1e-14
    # mirror x -> -x: velocity (vx, vy) -> (-vx, vy)
    vx, vy, _ = dvm.velocities()
    mir = [int(np.where((vx == -vx[i]) & (vy == vy[i]))[0][0]) for i in range(16)]
    fm = dvm.equilibrium(rho, -ux, uy, T, 2.0)
    assert np.abs(fm[mir] - f).max() < 1e-14
