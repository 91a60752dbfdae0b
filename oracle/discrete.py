"""The discrete operator on a periodic grid (oracle side).

Test infrastructure (see the package docstring).

Sec. 3.4 of the paper evaluates every cDFT integral as a discrete convolution
sum on the grid (its 1D example: h_k = sum_i f_i g_|k-i| dt).  That needs a
discrete kernel for each weight function.  The delta-shell weights have no
point values, so the kernel is defined spectrally: it is the inverse DFT of
the continuous transform sampled at the grid wave-vectors,

    K[m] = 1/(N h^3) sum_j w^(k_j) exp(+i k_j . r_m),   k_j = 2 pi j / (n h),

with the signed index j in [-n/2, n/2).  Consequences: h^3 sum_m K[m] = w^(0)
exactly (bulk sums are exact), and no r = 0 singularity appears for 1/r.

Nyquist reading (even n): a scalar weight depends on |k| only and takes
k = -pi/h on the Nyquist plane.  A vector weight -i k_hat_a V(|k|) is odd in
k_a, which the aliased Nyquist index cannot represent with a real kernel; its
a-component is set to zero where j_a = n/2 (other components are kept).

Orientation (Sec. 2.3.1): forward weighted densities are correlations,
n(r) = int rho(r') w(r' - r) dr'  ->  n^ = rho^ conj(w^);
back-convolutions are convolutions, mu(r) = int f(r') w(r - r') dr'  ->
mu^ = f^ w^.  The vector weight is taken outward, r_hat delta(|r| - R)
(the paper writes it as the gradient of its step function, whose sign would
point inward); mu is unchanged by flipping both vector weights together.

Pair kernels:
  MSA correlation (Sec. 2.3.4), per pair sigma = (d_i + d_j)/2,
    C_ij(r) = -q_i q_j l_B [2B/sigma - (B/sigma)^2 r - 1/r] for r <= sigma,
    B = [xi + 1 - sqrt(1 + 2 xi)]/xi = xi / (xi + 1 + sqrt(1 + 2 xi)),
    xi = kappa sigma.  (The printed prefactor e^2/(k_B T eps) is read as l_B.)
  square-well attraction (Sec. 2.3.2), u_ij(r) = -eps_ij on
    sigma_ij <= r <= r_out (r_out = gamma sigma_ij unless given); the hard
    core is left to the FMT term.
"""
from dataclasses import dataclass, field
import math
from typing import List, Optional

import numpy as np

from . import transforms as tr
from . import units


def signed_index(n: int) -> np.ndarray:
    j = np.arange(n)
    return np.where(j < n // 2, j, j - n) if n % 2 == 0 else np.where(j <= n // 2, j, j - n)


def wavevectors(n: int, h: float, half: bool = False):
    """Grid wave-vectors (kx, ky, kz) as broadcastable arrays, |k|, and the
    three unit-vector components with the Nyquist rule applied.
    half=True keeps only kz >= 0 (the numpy rfft layout)."""
    L = n * h
    jx = signed_index(n)
    jz = np.arange(n // 2 + 1) if half else signed_index(n)
    k1 = 2.0 * math.pi * jx / L
    kzv = 2.0 * math.pi * jz / L
    kx = k1[:, None, None]
    ky = k1[None, :, None]
    kz = kzv[None, None, :]
    kmag = np.sqrt(kx * kx + ky * ky + kz * kz)
    safe = np.where(kmag == 0.0, 1.0, kmag)
    khat = []
    for comp, idx, axis in ((kx, jx, 0), (ky, jx, 1), (kz, jz, 2)):
        u = comp / safe
        u = np.where(kmag == 0.0, 0.0, u)
        if n % 2 == 0:
            nyq = (np.abs(idx) == n // 2)
            shape = [1, 1, 1]
            shape[axis] = idx.shape[0]
            u = np.where(nyq.reshape(shape), 0.0, u)
        khat.append(np.broadcast_to(u, kmag.shape).copy())
    return kx, ky, kz, kmag, np.stack(khat)


@dataclass
class Operator:
    n: int
    h: float
    half: bool
    S: int
    kmag: np.ndarray
    khat: np.ndarray
    R: List[float]
    w: List[dict]
    beta: float
    lB: float
    kappa: float
    terms: int
    c_sw: float
    sigma: np.ndarray
    B: np.ndarray
    rout: np.ndarray
    eps: np.ndarray
    C_hat: Optional[list] = None     # [i][j] arrays, MSA transform (nm^3)
    u_hat: Optional[list] = None     # [i][j] arrays, well transform (eV nm^3)
    C0: Optional[np.ndarray] = None  # C_hat at k = 0
    mu_el_bulk: Optional[np.ndarray] = None
    rho_bulk: Optional[np.ndarray] = None

    @property
    def N(self):
        return self.n ** 3


def msa_B(xi: float) -> float:
    """B of the MSA correlation, xi = kappa sigma (Sec. 2.3.4)."""
    if xi == 0.0:
        return 0.0
    return xi / (xi + 1.0 + math.sqrt(1.0 + 2.0 * xi))


def build_operator(problem, half: bool = False) -> Operator:
    n, h = problem.n, problem.h
    sp = problem.species
    S = len(sp)
    _, _, _, kmag, khat = wavevectors(n, h, half)
    R = [0.5 * s.d for s in sp]
    w = []
    for Ri in R:
        j0 = tr.j0(kmag * Ri)
        v2 = tr.shell_vec_ft(kmag, Ri)
        w.append({
            "w0": j0,                                   # omega_2 / (4 pi R^2)
            "w1": Ri * j0,                              # omega_2 / (4 pi R)
            "w2": tr.shell_ft(kmag, Ri),                # delta(|r| - R)
            "w3": tr.ball_ft(kmag, Ri),                 # theta(R - |r|)
            "v2": v2,                                   # omega_2v = -i khat v2
            "v1": v2 / (4.0 * math.pi * Ri),            # omega_1v = omega_2v/(4 pi R)
        })
    b = units.beta(problem.T)
    lB = units.bjerrum_length(problem.T, problem.eps_r)
    k2 = units.kappa_squared(problem.T, problem.eps_r, [s.rho_bulk for s in sp], [s.q for s in sp])
    kappa = math.sqrt(k2)
    sigma = np.array([[0.5 * (sp[i].d + sp[j].d) for j in range(S)] for i in range(S)])
    B = np.array([[msa_B(kappa * sigma[i, j]) for j in range(S)] for i in range(S)])
    eps = np.zeros((S, S)) if problem.sw_eps is None else np.asarray(problem.sw_eps, float)
    rout = np.zeros((S, S)) if problem.sw_rout is None else np.asarray(problem.sw_rout, float)
    rout = np.where(rout > 0.0, rout, problem.sw_gamma * sigma)
    op = Operator(n=n, h=h, half=half, S=S, kmag=kmag, khat=khat, R=R, w=w, beta=b, lB=lB,
                  kappa=kappa, terms=problem.terms, c_sw=problem.sw_prefactor, sigma=sigma,
                  B=B, rout=rout, eps=eps,
                  mu_el_bulk=np.array([s.mu_el_bulk for s in sp]),
                  rho_bulk=np.array([s.rho_bulk for s in sp]))
    if problem.terms & 2:
        C_hat = [[None] * S for _ in range(S)]
        C0 = np.zeros((S, S))
        for i in range(S):
            for j in range(S):
                s_ij, B_ij = sigma[i, j], B[i, j]
                pref = -sp[i].q * sp[j].q * lB
                C_hat[i][j] = pref * (2.0 * B_ij / s_ij * tr.ball_ft(kmag, s_ij)
                                      - (B_ij / s_ij) ** 2 * tr.r_ball_ft(kmag, s_ij)
                                      - tr.inv_r_ball_ft(kmag, s_ij))
                C0[i, j] = pref * (2.0 * B_ij / s_ij * tr.ball_ft(0.0, s_ij)
                                   - (B_ij / s_ij) ** 2 * tr.r_ball_ft(0.0, s_ij)
                                   - tr.inv_r_ball_ft(0.0, s_ij))
        op.C_hat, op.C0 = C_hat, C0
    if problem.terms & 4:
        u_hat = [[None] * S for _ in range(S)]
        for i in range(S):
            for j in range(S):
                u_hat[i][j] = -eps[i, j] * (tr.ball_ft(kmag, rout[i, j])
                                            - tr.ball_ft(kmag, sigma[i, j]))
        op.u_hat = u_hat
    return op


def real_space_kernel(spec: np.ndarray, n: int, h: float) -> np.ndarray:
    """K[m] = 1/(N h^3) sum_j spec[j] exp(+2 pi i j.m / n), evaluated as three
    explicit DFT-matrix products (no FFT).  spec is on the full grid."""
    j = np.arange(n)
    E = np.exp(2j * math.pi * np.outer(j, j) / n)      # E[m, j]
    K = np.tensordot(E, spec, axes=([1], [0]))          # sum over jx
    K = np.tensordot(E, K, axes=([1], [1]))             # sum over jy -> (my, mx, jz)
    K = np.tensordot(E, K, axes=([1], [2]))             # sum over jz -> (mz, my, mx)
    K = np.transpose(K, (2, 1, 0)) / (n ** 3 * h ** 3)
    if np.max(np.abs(K.imag)) > 1e-9 * max(1.0, np.max(np.abs(K.real))):
        raise AssertionError("kernel spectrum is not Hermitian on the grid")
    return K.real.copy()
