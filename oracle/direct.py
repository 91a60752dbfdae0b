"""Direct O(N^2) periodic convolution sums (oracle side, no FFT).

Test infrastructure (see the package docstring).

Sec. 3.4 writes each cDFT integral as a discrete sum over grid points (its
1D example: h_k = sum_i f_i g_|k-i| dt).  On the periodic grid, with kernel
K and volume element h^3:

  correlation  out[r] = h^3 sum_r' f[r'] K[r' - r]     (forward weighted densities)
  convolution  out[r] = h^3 sum_r' f[r'] K[r - r']     (back-convolutions, pair terms)

indices taken modulo n per axis.  Each output point is one explicit sum over
all N input points; a stack of M (field, kernel) pairs is evaluated together.
"""
import numpy as np


def correlate_direct(F: np.ndarray, K: np.ndarray, h: float) -> np.ndarray:
    """F, K: (M, n, n, n).  out[m, r] = h^3 sum_r' F[m, r'] K[m, r' - r]."""
    F = np.asarray(F, dtype=np.float64)
    K = np.asarray(K, dtype=np.float64)
    M, n = F.shape[0], F.shape[1]
    out = np.empty_like(F)
    for rx in range(n):
        Kx = np.roll(K, rx, axis=1)                  # Kx[., i] = K[., i - rx]
        for ry in range(n):
            Kxy = np.roll(Kx, ry, axis=2)
            for rz in range(n):
                Kxyz = np.roll(Kxy, rz, axis=3)      # = K[., r' - r]
                out[:, rx, ry, rz] = np.einsum("mijk,mijk->m", F, Kxyz)
    return out * h ** 3


def reflect(K: np.ndarray) -> np.ndarray:
    """Kr[m] = K[-m mod n] on the last three axes."""
    Kr = K[..., ::-1, ::-1, ::-1]
    return np.roll(Kr, 1, axis=(-3, -2, -1))


def convolve_direct(F: np.ndarray, K: np.ndarray, h: float) -> np.ndarray:
    """out[m, r] = h^3 sum_r' F[m, r'] K[m, r - r']."""
    return correlate_direct(F, reflect(np.asarray(K, dtype=np.float64)), h)
