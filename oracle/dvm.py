"""D2V16 discrete-velocity model and its equilibrium (Sec. 2.1; Sec. 2.2, Chapman-Enskog
paragraph).  Test infrastructure only.

Velocity set: four rings of four velocities.  Ring 1 (i = 1..4, the only ring with eta_i =
eta0 = 2.5) and ring 3 (i = 9..12) lie on the axes, rings 2 and 5..8 and 4 (13..16) on the
diagonals; member k of a ring is rotated by k*90 degrees from member 0.  The paper takes the
ring speeds from Kataoka and Tsutahara without printing them: axis rings have velocities
(+-va, 0), (0, +-va) and (+-vc, 0), (0, +-vc); diagonal rings (+-vb, +-vb) and (+-vd, +-vd).

Equilibrium: the unique f^eq whose 16 discrete moments equal those of the Maxwellian with b
degrees of freedom -- the "seven kinetic moments": M0, M1, M2,0, M2, M3,1, M3 and M4,2
(1+2+1+3+2+4+3 = 16 scalar conditions).  With eta0 != 0 the 16x16 moment matrix is
invertible, so this equals any fourth-order polynomial equilibrium satisfying those moments.
"""
import numpy as np

DEFAULT_DVM = dict(va=1.0, vb=0.5, vc=2.0, vd=1.0, eta0=2.5)


def velocities(dvm=None):
    """Return vx[16], vy[16], eta[16] (population index 0..15 = paper i = 1..16)."""
    d = dict(DEFAULT_DVM)
    if dvm:
        d.update(dvm)
    axis = [(1.0, 0.0), (0.0, 1.0), (-1.0, 0.0), (0.0, -1.0)]
    diag = [(1.0, 1.0), (-1.0, 1.0), (-1.0, -1.0), (1.0, -1.0)]
    vx, vy = [], []
    for speed, unit in ((d["va"], axis), (d["vb"], diag), (d["vc"], axis), (d["vd"], diag)):
        for ex, ey in unit:
            vx.append(speed * ex)
            vy.append(speed * ey)
    eta = [d["eta0"]] * 4 + [0.0] * 12
    return np.array(vx), np.array(vy), np.array(eta)


def moment_matrix(vx, vy, eta):
    """Rows: the 16 moment weights [1, vx, vy, w, vx^2, vx vy, vy^2, w vx, w vy, vx^3, vx^2 vy,
    vx vy^2, vy^3, w vx^2, w vx vy, w vy^2] with w = v^2 + eta^2, evaluated at each velocity."""
    w = vx * vx + vy * vy + eta * eta
    rows = [np.ones_like(vx), vx, vy, w,
            vx * vx, vx * vy, vy * vy,
            w * vx, w * vy,
            vx ** 3, vx * vx * vy, vx * vy * vy, vy ** 3,
            w * vx * vx, w * vx * vy, w * vy * vy]
    return np.array(rows)


def maxwellian_moments(rho, ux, uy, T, b):
    """The seven kinetic moments of the Maxwellian with b degrees of freedom, in the row order
    of ``moment_matrix``.  Broadcasts over field arrays; returns shape (16, ...)."""
    u2 = ux * ux + uy * uy
    h2 = (b + 2.0) * T + u2          # enthalpy-like factor of M3,1 and M4,2
    h4 = (b + 4.0) * T + u2
    return np.array([
        rho,                                         # M0
        rho * ux, rho * uy,                          # M1
        rho * (b * T + u2),                          # M2,0
        rho * (T + ux * ux), rho * ux * uy, rho * (T + uy * uy),          # M2
        rho * ux * h2, rho * uy * h2,                                     # M3,1
        rho * (3.0 * T * ux + ux ** 3), rho * (T * uy + ux * ux * uy),    # M3
        rho * (T * ux + ux * uy * uy), rho * (3.0 * T * uy + uy ** 3),
        rho * (h2 * T + h4 * ux * ux), rho * h4 * ux * uy, rho * (h2 * T + h4 * uy * uy),  # M4,2
    ])


def equilibrium(rho, ux, uy, T, b, dvm=None):
    """f^eq[16, ...] solving moment_matrix @ f^eq = maxwellian_moments."""
    vx, vy, eta = velocities(dvm)
    C = moment_matrix(vx, vy, eta)
    M = maxwellian_moments(np.asarray(rho, float), np.asarray(ux, float),
                           np.asarray(uy, float), np.asarray(T, float), b)
    shape = M.shape[1:]
    f = np.linalg.solve(C, M.reshape(16, -1))
    return f.reshape((16,) + shape)
