"""Physical constants and the derived electrostatic scales (oracle side).

Test infrastructure (see the package docstring).

* beta = 1/(k_B T), Table 1 quotes it at T = 223 K in eV^-1.
* Bjerrum length l_B = e^2 / (4 pi eps_0 eps_r k_B T) (Sec. 2.3.3), Table 1
  quotes 4.514 nm at 223 K and eps_r = 16.6.
* Inverse Debye length: kappa^2 = e^2/(eps_0 eps_r k_B T) sum_i rho_i q_i^2
  (Sec. 2.3.4, the definition of xi), i.e. 4 pi l_B sum_i rho_i q_i^2.

Constants are the exact SI values (2019 redefinition) and CODATA 2018.
"""
import math

ELEMENTARY_CHARGE_C = 1.602176634e-19
VACUUM_PERMITTIVITY_F_PER_M = 8.8541878128e-12
BOLTZMANN_J_PER_K = 1.380649e-23

KB_EV_PER_K = BOLTZMANN_J_PER_K / ELEMENTARY_CHARGE_C
# e^2/(4 pi eps_0) expressed in eV * nm
COULOMB_EV_NM = (ELEMENTARY_CHARGE_C ** 2 / (4.0 * math.pi * VACUUM_PERMITTIVITY_F_PER_M)
                 / ELEMENTARY_CHARGE_C * 1e9)


def beta(T: float) -> float:
    """1/(k_B T) in eV^-1."""
    return 1.0 / (KB_EV_PER_K * T)


def bjerrum_length(T: float, eps_r: float) -> float:
    """l_B in nm."""
    return COULOMB_EV_NM / eps_r * beta(T)


def kappa_squared(T: float, eps_r: float, rho_bulk, q) -> float:
    """kappa^2 in nm^-2 from the bulk densities (nm^-3) and valences."""
    s = 0.0
    for r, z in zip(rho_bulk, q):
        s += r * z * z
    return 4.0 * math.pi * bjerrum_length(T, eps_r) * s
