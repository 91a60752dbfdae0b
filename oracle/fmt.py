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
