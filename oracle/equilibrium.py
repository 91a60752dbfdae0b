"""Equilibrium densities of the grand ensemble by Picard iteration (oracle side).

Test infrastructure (see the package docstring).

At equilibrium with the bulk reservoir (Sec. 3.2 solves for this state to
start the PNP iteration) every species satisfies

    rho_i(r) = rho_i^bulk exp(beta mu_i^bulk - beta mu_ex_i[rho](r) - beta V_i(r)),

with beta mu_i^bulk the excess chemical potential of the uniform bulk and
beta V_i an external potential.  Picard iteration with mixing lambda, as in
the relaxation of Sec. 3.2:

    rho <- (1 - lambda) rho + lambda rho^bulk exp(beta mu^bulk - beta mu_ex[rho] - beta V),

stopped when max_i max_r |rho_new - rho| / rho_i^bulk <= tol.  Stationary
species (Species.mobile false: the fixed sites of Sec. 2.3.2) keep their
densities; they still shape mu_ex of the others, and they are left out of
the residual.
"""
import numpy as np

from .mu_ex import mu_ex


def bulk_mu_ex(problem):
    """beta mu_ex of the uniform bulk state: the evaluation of uniform densities
    (an 8^3 grid suffices, the result does not depend on it)."""
    p8 = problem.with_(n=8)
    rho = np.stack([np.full((8, 8, 8), s.rho_bulk) for s in problem.species])
    return mu_ex(p8, rho, "fft")["total"][:, 0, 0, 0].copy()


def picard(problem, rho0, beta_v=None, lam=0.1, tol=1e-10, max_iter=200, mu_bulk=None):
    """Returns (rho, iterations, residual).  beta_v: [S][n][n][n] or None."""
    rho = np.array(rho0, dtype=np.float64)
    rb = np.array([s.rho_bulk for s in problem.species])
    mobile = [getattr(s, "mobile", True) for s in problem.species]
    mb = bulk_mu_ex(problem) if mu_bulk is None else np.asarray(mu_bulk, dtype=np.float64)
    res = np.inf
    for it in range(1, max_iter + 1):
        mu = mu_ex(problem, rho, "fft")["total"]
        new = rho.copy()
        res = 0.0
        for i in range(rho.shape[0]):
            if not mobile[i]:
                continue
            g = mb[i] - mu[i]
            if beta_v is not None:
                g = g - beta_v[i]
            new[i] = (1.0 - lam) * rho[i] + lam * rb[i] * np.exp(g)
            res = max(res, float(np.max(np.abs(new[i] - rho[i]) / rb[i])))
        rho = new
        if res <= tol:
            return rho, it, res
    return rho, max_iter, res
