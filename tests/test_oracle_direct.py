"""Pins for the direct sums: pure-Python loops of the defining formula on
tiny grids, orientation on a delta field, and agreement with the FFT route."""
import numpy as np
import pytest

import oracle
import pnp_inputs as P
from oracle.direct import correlate_direct, convolve_direct
from conftest import relerr


def _loops(F, K, h, sign):
    n = F.shape[0]
    out = np.zeros_like(F)
    for a in range(n):
        for b in range(n):
            for c in range(n):
                s = 0.0
                for i in range(n):
                    for j in range(n):
                        for k in range(n):
                            m = ((sign * (i - a)) % n, (sign * (j - b)) % n, (sign * (k - c)) % n)
                            s += F[i, j, k] * K[m]
                out[a, b, c] = s * h ** 3
    return out


@pytest.mark.parametrize("n", [3, 4])
def test_against_python_loops(n):
    rng = np.random.default_rng(n)
    F = rng.normal(size=(2, n, n, n))
    K = rng.normal(size=(2, n, n, n))
    h = 0.07
    c = correlate_direct(F, K, h)
    v = convolve_direct(F, K, h)
    for m in range(2):
        assert np.max(np.abs(c[m] - _loops(F[m], K[m], h, +1))) < 1e-13
        assert np.max(np.abs(v[m] - _loops(F[m], K[m], h, -1))) < 1e-13


def test_orientation_on_delta():
    n, h = 5, 1.0
    rng = np.random.default_rng(1)
    K = rng.normal(size=(1, n, n, n))
    F = np.zeros((1, n, n, n))
    F[0, 0, 0, 0] = 1.0
    c = correlate_direct(F, K, h)[0]
    v = convolve_direct(F, K, h)[0]
    for r in [(1, 2, 3), (4, 0, 1)]:
        neg = tuple((-x) % n for x in r)
        assert c[r] == pytest.approx(K[0][neg])     # K[r' - r] at r' = 0
        assert v[r] == pytest.approx(K[0][r])       # K[r - r'] at r' = 0


@pytest.mark.parametrize("maker", ["cfg1", "channel8", "channel12"])
def test_direct_route_equals_fft_route(maker):
    if maker == "cfg1":
        prob, rho = P.config1()
    elif maker == "channel8":
        prob, rho = P.channel_problem(8, 11)
    else:
        prob, rho = P.channel_problem(12, 12)
    a = oracle.mu_ex(prob, rho, "direct")
    b = oracle.mu_ex(prob, rho, "fft")
    for k in ("hs", "el", "sh", "total"):
        if np.max(np.abs(b[k])) > 0:
            assert relerr(a[k], b[k]) < 1e-12, k
