"""Rosenfeld fundamental-measure free-energy density and its derivatives.

Test infrastructure (see the package docstring).

Sec. 2.3.1 of the paper, the FMT form of Phi_hs (the first of its two
free-energy densities):

  Phi = -n0 ln(1 - n3) + n1 n2 / (1 - n3) + n2^3 / (24 pi (1 - n3)^2)
        - n1v.n2v / (1 - n3) - n2 (n2v.n2v) / (8 pi (1 - n3)^2)

and the ten partial derivatives the paper lists after the hard-sphere
chemical potential.  Vector arguments carry the component on axis 0.
"""
import math

import numpy as np


def _check_packing(n3):
    if np.any(n3 >= 1.0):
        raise ValueError("packing fraction n3 >= 1: ln(1 - n3) undefined")


def phi_hs(n0, n1, n2, n3, n1v, n2v):
    _check_packing(n3)
    one = 1.0 - n3
    v12 = np.sum(n1v * n2v, axis=0)
    v22 = np.sum(n2v * n2v, axis=0)
    return (-n0 * np.log1p(-n3) + n1 * n2 / one + n2 ** 3 / (24.0 * math.pi * one ** 2)
            - v12 / one - n2 * v22 / (8.0 * math.pi * one ** 2))


def dphi_hs(n0, n1, n2, n3, n1v, n2v):
    """Returns dict with d0, d1, d2, d3 (scalars) and d1v, d2v (3-vectors)."""
    _check_packing(n3)
    one = 1.0 - n3
    v12 = np.sum(n1v * n2v, axis=0)
    v22 = np.sum(n2v * n2v, axis=0)
    d0 = -np.log1p(-n3)
    d1 = n2 / one
    d2 = n1 / one + (n2 ** 2 - v22) / (8.0 * math.pi * one ** 2)
    d3 = (n0 / one + (n1 * n2 - v12) / one ** 2
          + (n2 ** 3 - 3.0 * n2 * v22) / (12.0 * math.pi * one ** 3))
    d1v = n2v / (n3 - 1.0)
    d2v = n1v / (n3 - 1.0) - n2 * n2v / (4.0 * math.pi * one ** 2)
    return {"d0": d0, "d1": d1, "d2": d2, "d3": d3, "d1v": d1v, "d2v": d2v}


# ---------------------------------------------------------------------------
# The modified (White Bear) form, the second free-energy density of Sec. 2.3.1:
#
#   Phi = -n0 ln(1 - n3) + (n1 n2 - n1v.n2v) / (1 - n3)
#         + (n2^3 - 3 n2 n2v.n2v) phi3(n3),
#   phi3(x) = [x + (1 - x)^2 ln(1 - x)] / (36 pi x^2 (1 - x)^2)
#           = [ln(1 - x) / (36 pi x^2) + 1 / (36 pi x (1 - x)^2)],
#
# the printed bracket of the n2^3 term, and -3 times it for the vector term.
# phi3 -> 1/(24 pi) as x -> 0 (the Rosenfeld value).  For small x the closed
# form cancels; its power series  36 pi phi3(x) = sum_k (k+1)(k+3)/(k+2) x^k
# (from ln(1 - x) = -sum x^k / k) is used below x = 0.05.
# ---------------------------------------------------------------------------
WB_SERIES_BELOW = 0.05


def _wb_g(x):
    """g(x) = 36 pi phi3(x) and g'(x)."""
    x = np.asarray(x, dtype=np.float64)
    small = np.abs(x) < WB_SERIES_BELOW
    xs = np.where(small, x, 0.0)
    g_s = np.zeros_like(x)
    dg_s = np.zeros_like(x)
    for k in range(16):
        c = (k + 1) * (k + 3) / (k + 2)
        g_s = g_s + c * xs ** k
        if k > 0:
            dg_s = dg_s + k * c * xs ** (k - 1)
    xl = np.where(small, 0.5, x)
    one = 1.0 - xl
    ln = np.log1p(-xl)
    num = xl + one ** 2 * ln
    g_l = num / (xl ** 2 * one ** 2)
    dnum = xl - 2.0 * one * ln
    dg_l = (dnum * xl * one - 2.0 * num * (1.0 - 2.0 * xl)) / (xl ** 3 * one ** 3)
    return np.where(small, g_s, g_l), np.where(small, dg_s, dg_l)


def phi_hs_wb(n0, n1, n2, n3, n1v, n2v):
    _check_packing(n3)
    one = 1.0 - n3
    v12 = np.sum(n1v * n2v, axis=0)
    v22 = np.sum(n2v * n2v, axis=0)
    g, _ = _wb_g(n3)
    return (-n0 * np.log1p(-n3) + (n1 * n2 - v12) / one
            + (n2 ** 3 - 3.0 * n2 * v22) * g / (36.0 * math.pi))


def dphi_hs_wb(n0, n1, n2, n3, n1v, n2v):
    """Derivatives of the White Bear Phi (same keys as dphi_hs)."""
    _check_packing(n3)
    one = 1.0 - n3
    v12 = np.sum(n1v * n2v, axis=0)
    v22 = np.sum(n2v * n2v, axis=0)
    g, dg = _wb_g(n3)
    p3, dp3 = g / (36.0 * math.pi), dg / (36.0 * math.pi)
    d0 = -np.log1p(-n3)
    d1 = n2 / one
    d2 = n1 / one + 3.0 * (n2 ** 2 - v22) * p3
    d3 = n0 / one + (n1 * n2 - v12) / one ** 2 + (n2 ** 3 - 3.0 * n2 * v22) * dp3
    d1v = n2v / (n3 - 1.0)
    d2v = n1v / (n3 - 1.0) - 6.0 * n2 * n2v * p3
    return {"d0": d0, "d1": d1, "d2": d2, "d3": d3, "d1v": d1v, "d2v": d2v}
