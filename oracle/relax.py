"""Density update of the consumer stub (oracle side).

Test infrastructure (see the package docstring).

Between two evaluations of mu_ex a PNP loop changes the densities.  Here the
change is a relaxation toward the equilibrium of the current excess chemical
potential: the equilibrium density of species i in the grand ensemble is
rho_i^bulk exp(beta mu_i^bulk - beta mu_ex_i(r)) (no potential, no ideal-gas
constant beyond the bulk reference), and the new density mixes it with the
old one as the relaxation step of Sec. 3.2 mixes new and old iterates:

    rho_i <- (1 - lambda) rho_i + lambda rho_i^bulk exp(g_i),
    g_i = beta mu_i^bulk - beta mu_ex_i, limited to [-clip, clip] when clip > 0.

The limit is this build's choice for the stub (the paper's PNP loop has no
such step): it bounds every density by max(rho_i, e^clip rho_i^bulk).

Stationary species (the fixed sites of Sec. 2.3.2, which are not transported)
keep their densities.
"""
import numpy as np


def relax_densities(rho, mu_ex, rho_bulk, mu_bulk, lam, clip=0.0, mobile=None):
    """rho, mu_ex: float64 [S][...]; rho_bulk, mu_bulk: S values; lam in [0, 1];
    mobile: S flags (None: every species moves)."""
    rho = np.asarray(rho, dtype=np.float64)
    mu_ex = np.asarray(mu_ex, dtype=np.float64)
    out = np.empty_like(rho)
    for i in range(rho.shape[0]):
        if mobile is not None and not mobile[i]:
            out[i] = rho[i]
            continue
        g = mu_bulk[i] - mu_ex[i]
        if clip > 0:
            g = np.clip(g, -clip, clip)
        target = rho_bulk[i] * np.exp(g)
        out[i] = (1.0 - lam) * rho[i] + lam * target
    return out
