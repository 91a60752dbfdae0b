"""Pins for the continuous radial transforms: numerical quadrature of the
defining radial integrals with scipy's spherical Bessel functions."""
import math

import numpy as np
import pytest
from scipy import integrate, special

from oracle import transforms as tr

KS = [0.0, 1e-4, 0.3, 2.0, 3.7, 7.9, 19.0, 55.0]


def radial_ft(f, a, k):
    """4 pi int_0^a f(r) r^2 j0(k r) dr by adaptive quadrature."""
    g = lambda r: f(r) * r * r * special.spherical_jn(0, k * r)
    val, _ = integrate.quad(g, 0.0, a, limit=400, epsabs=0.0, epsrel=1e-13)
    return 4.0 * math.pi * val


@pytest.mark.parametrize("a", [0.075, 0.15, 0.3, 0.6])
@pytest.mark.parametrize("k", KS)
def test_ball(a, k):
    ref = radial_ft(lambda r: 1.0, a, k)
    assert tr.ball_ft(k, a) == pytest.approx(ref, rel=1e-11, abs=1e-14 * a ** 3)


@pytest.mark.parametrize("a", [0.15, 0.3])
@pytest.mark.parametrize("k", KS)
def test_r_ball(a, k):
    ref = radial_ft(lambda r: r, a, k)
    assert tr.r_ball_ft(k, a) == pytest.approx(ref, rel=1e-11, abs=1e-14 * a ** 4)


@pytest.mark.parametrize("a", [0.15, 0.3])
@pytest.mark.parametrize("k", KS)
def test_inv_r_ball(a, k):
    # the integrand r^2 j0 / r is regular at 0
    g = lambda r: r * special.spherical_jn(0, k * r)
    val, _ = integrate.quad(g, 0.0, a, limit=400, epsabs=0.0, epsrel=1e-13)
    assert tr.inv_r_ball_ft(k, a) == pytest.approx(4 * math.pi * val, rel=1e-11, abs=1e-15)


@pytest.mark.parametrize("a", [0.075, 0.2])
@pytest.mark.parametrize("k", KS)
def test_shell_is_derivative_of_ball(a, k):
    # d/da theta(a - r) = delta(r - a): the shell transform is d/da of the ball's
    da = 1e-5 * a
    fd = (tr.ball_ft(k, a + da) - tr.ball_ft(k, a - da)) / (2 * da)
    assert tr.shell_ft(k, a) == pytest.approx(fd, rel=1e-8, abs=1e-12)


@pytest.mark.parametrize("a", [0.075, 0.2])
@pytest.mark.parametrize("k", KS)
def test_vector_shell_radial_part(a, k):
    # int r_hat delta(r - a) e^{-ik.r} = -i k_hat 4 pi a^2 j1(k a)
    ref = 4 * math.pi * a * a * special.spherical_jn(1, k * a)
    assert tr.shell_vec_ft(k, a) == pytest.approx(ref, rel=1e-12, abs=1e-16)


def test_series_switch_is_continuous():
    for f, x0 in ((tr.j1_over_x, 0.5), ):
        lo, hi = f(np.nextafter(x0, 0.0)), f(x0)
        assert abs(lo - hi) < 1e-15
    y0 = 1.0
    lo, hi = tr.r_ball_ft(np.nextafter(y0, 0.0), 1.0), tr.r_ball_ft(y0, 1.0)
    assert abs(lo - hi) / abs(hi) < 1e-14
