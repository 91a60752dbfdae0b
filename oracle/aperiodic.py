"""Aperiodic (zero-extension) evaluation of beta mu_ex (oracle side).

Test infrastructure (see the package docstring).

Sec. 3.4 evaluates each convolution integral over the computational domain
only, int_Omega f(r') g(|r - r'|) dr', by extending the sampled integrand with
zeros to twice the grid length per axis and taking circular convolutions of
that doubled length; Sec. 3.5 states the same zero extension for the delta
shells that leave the domain.  Here:

  * the domain Omega is the n^3 grid, placed at the corner of a (2n)^3 grid
    of the same spacing;
  * every integrand is zero outside Omega: rho for the hard-sphere weights
    and the square well, rho - rho_bulk for the electrostatic correlation,
    and dPhi/dn_alpha for the hard-sphere back-convolution;
  * the discrete kernels are the spectral ones of the (2n)^3 grid, and the
    result is the periodic operator of that grid applied to the extended
    fields, read back on Omega.

Displacements between two points of Omega stay below n per axis, so no
pair of domain points meets through the doubled period: every convolution
is exactly the finite sum over Omega with the kernel of the doubled grid
(pinned against those sums written out).  Sec. 2.3.1 integrates the
hard-sphere free-energy density over Omega, F_hs = int_Omega Phi(n(r)) dr,
and its chemical potential mu_hs(r') = sum_alpha int_Omega dPhi/dn_alpha(r)
omega_alpha(r' - r) dr.  The weighted densities themselves are non-zero
outside Omega (a sphere centred outside still overlaps the domain), but
Phi is not integrated there, so the derivative fields are set to zero
outside Omega before the back-convolution (pinned by finite differences of
F_hs = h^3 sum_Omega Phi).

The 1D construction of Sec. 3.4 (two auxiliary kernel vectors, one reflected)
is restated in `split_convolution_1d`; its reflected vector as printed is
off by one (see `split_convolution_1d`).
"""
import numpy as np

from .mu_ex import mu_ex


def extend(field, n2):
    """Zero extension of [..., n, n, n] to [..., n2, n2, n2] (domain at the corner)."""
    field = np.asarray(field, dtype=np.float64)
    n = field.shape[-1]
    out = np.zeros(field.shape[:-3] + (n2, n2, n2))
    out[..., :n, :n, :n] = field
    return out


def mu_ex_aperiodic(problem, rho, route="fft"):
    """Per-term beta mu_ex and the Slotboom factor on Omega (keys as mu_ex),
    plus 'n_ext' (the weighted densities on the doubled grid, or None)."""
    rho = np.asarray(rho, dtype=np.float64)
    n = rho.shape[1]
    n2 = 2 * n
    rb = np.array([s.rho_bulk for s in problem.species])
    big = problem.with_(n=n2)
    domain = np.zeros((n2, n2, n2), dtype=bool)
    domain[:n, :n, :n] = True
    res = mu_ex(big, extend(rho, n2), route, drho=extend(rho - rb[:, None, None, None], n2), domain=domain)
    out = {k: res[k][:, :n, :n, :n].copy() for k in ("hs", "el", "sh", "total", "slotboom")}
    out["n_ext"] = res["n"]
    return out


def linear_convolution_1d(f, g):
    """h_k = sum_{i=0}^{N-1} f_i g_|k-i|, k = 0..N-1 (the trapezoidal sum of
    Sec. 3.4 with equal end values), by its definition."""
    N = len(f)
    return np.array([sum(f[i] * g[abs(k - i)] for i in range(N)) for k in range(N)])


def split_convolution_1d(f, g, shift=1):
    """The same sum through two circular convolutions of length 2N (Sec. 3.4):
    f^ = f zero-extended, g^ = g zero-extended, g~_i = g_(N-1-i) for
    0 <= i <= N-2 (else 0); then h_k = (f^ * g^)_k + (f^ * g~)_(k+N-1).
    shift=1 is that reflected index; shift=2 gives the printed g_(N-2-i),
    which shifts the second sum by one place (kept to document the reading).
    The circular convolutions are written out as sums (no FFT)."""
    f = np.asarray(f, dtype=np.float64)
    g = np.asarray(g, dtype=np.float64)
    N = len(f)
    M = 2 * N
    fh = np.zeros(M); fh[:N] = f
    gh = np.zeros(M); gh[:N] = g
    gt = np.zeros(M)
    for i in range(N - 1):
        gt[i] = g[N - shift - i] if 0 <= N - shift - i < N else 0.0

    def circ(a, b, k):
        return sum(a[i] * b[(k - i) % M] for i in range(M))

    return np.array([circ(fh, gh, k) + circ(fh, gt, k + N - 1) for k in range(N)])
