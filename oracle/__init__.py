"""CPU FP64 oracle for the cDFT excess chemical potential (TEST INFRASTRUCTURE).

This package is test infrastructure.  Only the tests, the smoke check and the
CPU-baseline leg of the benchmark may import or run it; the product path (the
HIP library and its Python binding) never touches it, and it shares no code
with that path.  Everything here is plain numpy/scipy in float64, written to
be checked against the paper by eye rather than to be fast.

What it computes (paper Sec. 2.3 and Sec. 3.4): for S species with densities
rho_i on a periodic n^3 grid of spacing h,

  * the FMT weighted densities n_0..n_3, n_1v, n_2v  (Sec. 2.3.1),
  * the ten partial derivatives of the Rosenfeld free-energy density (or of
    the modified White Bear form),
  * the hard-sphere chemical potential by back-convolution (Sec. 2.3.1),
  * the MSA electrostatic-correlation term (Sec. 2.3.4),
  * the mean-field square-well term (Sec. 2.3.2),
  * beta*mu_ex and the Slotboom factor exp(-beta*mu_ex) (Sec. 2.1).

The delta-shell integrals can also be taken by the product quadrature over
spheres of Sec. 3.5 (``shell_integrals``), with the smoothed-delta
alternative beside it for comparison.

An aperiodic mode (``mu_ex_aperiodic``: integrands zero outside the domain,
convolutions on the doubled grid, Sec. 3.4) sits on top of the periodic
operator.

Two evaluation routes of the same discrete operator are provided:
``direct`` (O(N^2) real-space sums with kernels built by an explicit inverse
DFT, no FFT anywhere) and ``fft`` (numpy FFTs as a library primitive).

Parity status per function is listed in ``oracle.STATUS``; every function is
pinned by a test against closed forms, invariants or brute force (see the
tests named there).
"""
from .units import beta, bjerrum_length, kappa_squared, KB_EV_PER_K, COULOMB_EV_NM
from .transforms import (ball_ft, shell_ft, shell_vec_ft, r_ball_ft, inv_r_ball_ft,
                         j0, j1, j1_over_x)
from .discrete import (Operator, build_operator, real_space_kernel, wavevectors)
from .fmt import phi_hs, dphi_hs, phi_hs_wb, dphi_hs_wb
from .direct import correlate_direct, convolve_direct
from .mu_ex import mu_ex, weighted_densities, free_energy
from .relax import relax_densities
from .equilibrium import picard, bulk_mu_ex
from .aperiodic import mu_ex_aperiodic, extend, linear_convolution_1d, split_convolution_1d
from .sphere_quad import (sphere_rule, shell_integrals, shell_integrals_at, shell_weighted_densities,
                          gaussian_bump_shell, shell_integral_gaussian_delta)

STATUS = {
    "units": "pinned: tests/test_oracle_units.py (Table 1 beta and l_B)",
    "transforms": "pinned: tests/test_oracle_transforms.py (radial quadrature)",
    "discrete": "pinned: tests/test_oracle_discrete.py (bulk sums, plane waves, realness)",
    "fmt": "pinned: tests/test_oracle_fmt.py (finite differences of Phi, PY bulk)",
    "direct": "pinned: tests/test_oracle_direct.py (brute-force loops, FFT route)",
    "mu_ex": "pinned: tests/test_oracle_mu_ex.py (bulk closed forms, FD consistency, symmetry)",
    "relax": "pinned: tests/test_oracle_relax.py (lambda 0 and 1, bulk fixed point)",
    "equilibrium": "pinned: tests/test_oracle_equilibrium.py (bulk fixed point, dilute Boltzmann limit, self-consistency)",
    "aperiodic": "pinned: tests/test_oracle_aperiodic.py (1D trapezoidal sum, domain sums of the linear terms, "
                 "direct route, mirror covariance)",
    "sphere_quad": "pinned: tests/test_oracle_sphere_quad.py (constant and affine fields, Gaussian bump closed "
                   "form at O(h^2), quarter turn, zero extension vs padded periodic grid, uniform-fluid FMT values)",
}

__all__ = [
    "beta", "bjerrum_length", "kappa_squared", "KB_EV_PER_K", "COULOMB_EV_NM",
    "ball_ft", "shell_ft", "shell_vec_ft", "r_ball_ft", "inv_r_ball_ft", "j0", "j1",
    "j1_over_x", "Operator", "build_operator", "real_space_kernel", "wavevectors",
    "phi_hs", "dphi_hs", "phi_hs_wb", "dphi_hs_wb", "correlate_direct", "convolve_direct", "mu_ex",
    "weighted_densities", "free_energy", "relax_densities", "picard", "bulk_mu_ex", "mu_ex_aperiodic",
    "extend", "linear_convolution_1d", "split_convolution_1d", "sphere_rule", "shell_integrals", "shell_integrals_at",
    "shell_weighted_densities", "gaussian_bump_shell", "shell_integral_gaussian_delta", "STATUS",
]
