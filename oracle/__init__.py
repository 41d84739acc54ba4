"""FP64 CPU oracle for the D2V16 windowed-FFT thermal liquid-vapour lattice Boltzmann step.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or link this package:
only the tests, the smoke check and the benchmark's CPU-baseline leg use it.  It shares no code,
tables or constants with the HIP library; the two meet only through the seeded input arrays.

The oracle follows Gan, Xu, Zhang, Wang, Yu, Yang, "Lattice Boltzmann kinetic modeling and
simulation of thermal liquid-vapor system" (arXiv 1403.3746):

* ``dvm``       -- D2V16 velocity set, the seven kinetic moments and the equilibrium
                   (Sec. 2.1 and the Chapman-Enskog paragraph of Sec. 2.2).
* ``spectral``  -- the windowed-FFT derivative, Eq. (3) (Sec. 2.3).
* ``eos``       -- van der Waals pressure, chemical potential and Maxwell construction
                   (Sec. 2.2 NS system; Sec. 3.1 and 3.3).
* ``model``     -- moments, forcing term I_i (Eq. 2), right-hand side of Eq. (1), the two-stage
                   Runge-Kutta step (Sec. 2.3) and the total-energy diagnostic (Sec. 2.2).

Everything is plain NumPy/SciPy in float64 with no blocking or fusion.  Pins that tie each
function to something other than itself live in ``tests/test_oracle_*.py``.  Parity status:
every function is pinned.  B, C and C_q on general non-uniform fields (T, u and rho all varying,
H, zeta, q != 0) and the total energy e_T are pinned against the paper's formulas differentiated
and integrated exactly (sympy) on band-limited fields, with negative controls for the plausible
slips; the rest against closed forms, identities, special cases and a naive DFT.
"""
