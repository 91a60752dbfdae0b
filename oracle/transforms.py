"""Continuous Fourier transforms of the radial kernels (oracle side).

Test infrastructure (see the package docstring).

Convention: f^(k) = integral f(r) exp(-i k.r) d^3r.  For a radial f this is
4 pi int_0^inf f(r) r^2 j0(k r) dr; for a radial vector field f(r) r_hat it is
-i k_hat 4 pi int_0^inf f(r) r^2 j1(k r) dr.

Kernels needed by the method (Sec. 2.3.1 weight functions, Sec. 2.3.2 square
well, Sec. 2.3.4 MSA correlation), all with x = k a:

  ball      theta(a - r)          4 pi a^3 j1(x)/x
  shell     delta(r - a)          4 pi a^2 j0(x)
  vec shell r_hat delta(r - a)    -i k_hat 4 pi a^2 j1(x)   (radial part returned)
  r-ball    r theta(a - r)        4 pi a^4 [2 x sin x + (2 - x^2) cos x - 2] / x^4
  1/r-ball  theta(a - r) / r      4 pi a^2 (1 - cos x) / x^2 = 4 pi a^2 * 2 sin^2(x/2)/x^2

Closed forms lose digits to cancellation at small x; there the Taylor series
of the defining integrals are used instead:
  j1(x)/x   = sum_m (-1)^m x^(2m) / ((2m+1)! (2m+3))
  r-ball/(4 pi a^4) = sum_m (-1)^m x^(2m) / ((2m+1)! (2m+4))
"""
import math

import numpy as np

_J1X_SWITCH = 0.5
_RB_SWITCH = 1.0


def _series(x2, denom_offset, terms):
    out = np.zeros_like(x2)
    p = np.ones_like(x2)
    for m in range(terms):
        out = out + ((-1) ** m) * p / (math.factorial(2 * m + 1) * (2 * m + denom_offset))
        p = p * x2
    return out


def j0(x):
    x = np.asarray(x, dtype=np.float64)
    safe = np.where(x == 0.0, 1.0, x)
    return np.where(x == 0.0, 1.0, np.sin(safe) / safe)


def j1_over_x(x):
    x = np.asarray(x, dtype=np.float64)
    small = np.abs(x) < _J1X_SWITCH
    safe = np.where(small, 1.0, x)
    closed = (np.sin(safe) - safe * np.cos(safe)) / safe ** 3
    return np.where(small, _series(x * x, 3, 8), closed)


def j1(x):
    x = np.asarray(x, dtype=np.float64)
    return x * j1_over_x(x)


def ball_ft(k, a):
    """Transform of the unit ball of radius a (weight omega_3)."""
    return 4.0 * math.pi * a ** 3 * j1_over_x(np.asarray(k) * a)


def shell_ft(k, a):
    """Transform of the spherical shell delta(r - a) (weight omega_2)."""
    return 4.0 * math.pi * a ** 2 * j0(np.asarray(k) * a)


def shell_vec_ft(k, a):
    """Radial part V of the transform of r_hat delta(r - a): the full
    transform is -i k_hat V(k)."""
    return 4.0 * math.pi * a ** 2 * j1(np.asarray(k) * a)


def r_ball_ft(k, a):
    """Transform of r * theta(a - r)."""
    y = np.asarray(k, dtype=np.float64) * a
    small = np.abs(y) < _RB_SWITCH
    s = np.where(small, 1.0, y)
    closed = (2.0 * s * np.sin(s) + (2.0 - s * s) * np.cos(s) - 2.0) / s ** 4
    return 4.0 * math.pi * a ** 4 * np.where(small, _series(y * y, 4, 10), closed)


def inv_r_ball_ft(k, a):
    """Transform of theta(a - r) / r."""
    y = np.asarray(k, dtype=np.float64) * a
    s = np.where(y == 0.0, 1.0, y)
    f = np.where(y == 0.0, 0.5, 2.0 * np.sin(0.5 * s) ** 2 / (s * s))
    return 4.0 * math.pi * a ** 2 * f
