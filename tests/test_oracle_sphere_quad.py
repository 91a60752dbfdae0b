"""Pins of the sphere-quadrature oracle (Sec. 3.5) against closed forms and invariants.

Each check fixes a different part of the product rule: the constant field
fixes R^2, the sin(phi) Jacobian and the 1D weights; the affine field fixes
the interpolation and the axis order of the node directions (and the sign and
R^3 scale of the vector integral); the Gaussian bump fixes everything against
an elementary closed form and shows the trilinear O(h^2) rate; the quarter
turn fixes the orientation of theta and the vector components; the padded
grid fixes the zero extension.
"""
import math

import numpy as np
import pytest

from oracle import sphere_quad as Q


def test_rule_integrates_sphere_area():
    for k in (6, 8, 12):
        th, wt, ph, wp = Q.sphere_rule(k)
        area = np.sum(wt) * np.sum(wp * np.sin(ph))
        assert abs(area - 4.0 * math.pi) < 1e-9 * 4.0 * math.pi
        assert np.all((ph > 0.0) & (ph < math.pi))
        assert th[0] == 0.0 and abs(th[1] - 2.0 * math.pi / k) < 1e-15


@pytest.mark.parametrize("aperiodic", [False, True])
def test_constant_field(aperiodic):
    n, h, R, c = 10, 0.1, 0.37, 2.5
    f = np.full((n, n, n), c)
    I, Iv = Q.shell_integrals(f, R, h, 8, aperiodic=aperiodic)
    exact = 4.0 * math.pi * R * R * c
    inner = (slice(5, 6),) * 3 if aperiodic else (slice(None),) * 3
    assert np.max(np.abs(I[inner] - exact)) < 1e-12 * exact
    assert np.max(np.abs(Iv[(slice(None),) + inner])) < 1e-12 * exact


def test_affine_field_interior():
    n, h, R = 16, 0.1, 0.37          # R/h = 3.7: nodes fall between grid points
    a = 0.8
    b = np.array([0.3, -0.7, 1.1])
    x = h * np.arange(n)
    X, Y, Z = np.meshgrid(x, x, x, indexing="ij")
    f = a + b[0] * X + b[1] * Y + b[2] * Z
    # order 12: the polar rule's own error on int sin^3 and int cos^2 sin is below 1e-13 there
    I, Iv = Q.shell_integrals(f, R, h, 12, aperiodic=True)
    lo, hi = 5, n - 5                # spheres of radius 3.7 h stay inside the grid
    s = (slice(lo, hi),) * 3
    ref = 4.0 * math.pi * R * R * f[s]
    assert np.max(np.abs(I[s] - ref)) < 1e-11 * np.max(np.abs(ref))
    for ax in range(3):
        # R^2 int (a + b.(r + R n)) n_ax dOmega = R^3 b_ax 4 pi / 3
        want = 4.0 * math.pi / 3.0 * R ** 3 * b[ax]
        assert np.max(np.abs(Iv[ax][s] - want)) < 1e-11 * 4.0 * math.pi * R ** 3


def test_cubic_weights_reproduce_cubics():
    # the tricubic interpolant is exact for every polynomial of degree <= 3 per axis
    # (a wrong Lagrange coefficient breaks one of these monomials)
    rng = np.random.default_rng(11)
    n = 12
    i = np.arange(n, dtype=np.float64)
    X, Y, Z = np.meshgrid(i, i, i, indexing="ij")
    s = (slice(3, n - 3),) * 3
    for px, py, pz in ((3, 0, 0), (0, 3, 0), (0, 0, 3), (2, 1, 3), (1, 1, 1), (0, 2, 2)):
        f = X ** px * Y ** py * Z ** pz
        for _ in range(3):
            p = rng.uniform(-2.0, 2.0, size=3)
            g = Q.interpolate_shifted(f, p, aperiodic=True, cubic=True)
            want = (X + p[0]) ** px * (Y + p[1]) ** py * (Z + p[2]) ** pz
            assert np.max(np.abs(g[s] - want[s])) < 1e-10 * np.max(np.abs(want[s])), (px, py, pz, p)
    # and, unlike the trilinear one, it is not exact for degree 4
    f = X ** 4
    g = Q.interpolate_shifted(f, (0.5, 0.0, 0.0), aperiodic=True, cubic=True)
    assert np.max(np.abs(g[s] - ((X + 0.5) ** 4)[s])) > 1e-3


def test_cubic_field_interior_closed_form():
    # f = x^3: R^2 int (x + R n_x)^3 dOmega = 4 pi R^2 (x^3 + x R^2), and the
    # x component of the vector integral R^2 int (x + R n_x)^3 n_x dOmega =
    # 4 pi R^3 x^2 + 4 pi R^5 / 5; the y and z components vanish
    n, h, R = 18, 0.1, 0.37
    x = h * np.arange(n)
    X = np.meshgrid(x, x, x, indexing="ij")[0]
    f = X ** 3
    pts = np.array([[a, b, c] for a in (7, 9, 10) for b in (6, 8) for c in (7, 11)])
    I, Iv = Q.shell_integrals_at(f, R, h, 24, pts, aperiodic=True, cubic=True)
    xs = h * pts[:, 0]
    ref = 4.0 * math.pi * R * R * (xs ** 3 + xs * R * R)
    assert np.max(np.abs(I - ref)) < 1e-9 * np.max(np.abs(ref))
    refv = 4.0 * math.pi * R ** 3 * xs ** 2 + 4.0 * math.pi * R ** 5 / 5.0
    assert np.max(np.abs(Iv[0] - refv)) < 1e-9 * np.max(np.abs(refv))
    assert np.max(np.abs(Iv[1:])) < 1e-9 * np.max(np.abs(refv))
    # the trilinear interpolant misses the curvature
    I1, _ = Q.shell_integrals_at(f, R, h, 24, pts, aperiodic=True)
    assert np.max(np.abs(I1 - ref)) > 1e-4 * np.max(np.abs(ref))


def _bump_errors(n, k=16, cubic=False):
    L, s, R = 4.8, 0.3, 0.25
    h = L / n
    x = h * np.arange(n)
    c = np.array([L / 2, L / 2 + 0.5 * h, L / 2 - 0.3 * h])   # centre off the grid
    X, Y, Z = np.meshgrid(x, x, x, indexing="ij")
    D = np.stack([X - c[0], Y - c[1], Z - c[2]])
    d = np.sqrt(np.sum(D * D, axis=0))
    f = np.exp(-d * d / (2.0 * s * s))
    I, Iv = Q.shell_integrals(f, R, h, k, cubic=cubic)
    I_ex, Ir_ex = Q.gaussian_bump_shell(d, R, s)
    Iv_ex = Ir_ex * D / np.where(d > 0, d, 1.0)
    e_s = np.max(np.abs(I - I_ex)) / np.max(np.abs(I_ex))
    e_v = np.max(np.abs(Iv - Iv_ex)) / np.max(np.abs(Ir_ex))
    return e_s, e_v


def test_gaussian_bump_closed_form_second_order():
    e1s, e1v = _bump_errors(24)
    e2s, e2v = _bump_errors(48)
    # bump width 1.5 h on the coarse grid: the trilinear error is 7 % (scalar) and 11 % (vector)
    # of the largest value there, and a quarter of that at h / 2
    assert e1s < 0.1 and e1v < 0.15
    assert e2s < 0.025 and e2v < 0.04
    assert 3.0 < e1s / e2s < 5.5, (e1s, e2s)
    assert 3.0 < e1v / e2v < 5.5, (e1v, e2v)


def test_gaussian_bump_cubic_fourth_order():
    # with the tricubic interpolant the error falls as h^4: far below the
    # trilinear one, and by about 16 when h halves
    e1s, e1v = _bump_errors(24, cubic=True)
    e2s, e2v = _bump_errors(48, cubic=True)
    t1s, _ = _bump_errors(24)
    assert e1s < 0.25 * t1s
    assert 9.0 < e1s / e2s < 25.0, (e1s, e2s)
    assert 9.0 < e1v / e2v < 25.0, (e1v, e2v)


def test_bump_closed_form_small_distance_limit():
    R, s = 0.25, 0.3
    I0, Iv0 = Q.gaussian_bump_shell(np.array([0.0, 1e-9]), R, s)
    assert abs(I0[0] - 4.0 * math.pi * R * R * math.exp(-R * R / (2 * s * s))) < 1e-14
    assert abs(I0[1] - I0[0]) < 1e-12 and abs(Iv0[0]) < 1e-14


def test_quarter_turn_about_z():
    rng = np.random.default_rng(5)
    n, h, R = 9, 0.1, 0.26
    f = rng.random((n, n, n))
    # f'(r) = f(Q^-1 r) with Q (x, y, z) = (-y, x, z): f'[i, j, l] = f[j, -i, l]
    fr = np.roll(f.transpose(1, 0, 2)[::-1], 1, axis=0)
    I, Iv = Q.shell_integrals(f, R, h, 8)
    Ir, Ivr = Q.shell_integrals(fr, R, h, 8)

    def rot(g):
        return np.roll(g.transpose(1, 0, 2)[::-1], 1, axis=0)

    assert np.max(np.abs(Ir - rot(I))) < 1e-12
    assert np.max(np.abs(Ivr[0] + rot(Iv[1]))) < 1e-12
    assert np.max(np.abs(Ivr[1] - rot(Iv[0]))) < 1e-12
    assert np.max(np.abs(Ivr[2] - rot(Iv[2]))) < 1e-12


def test_zero_extension_equals_padded_periodic():
    rng = np.random.default_rng(6)
    n, h, R, pad = 7, 0.1, 0.23, 4
    f = rng.random((n, n, n))
    big = np.zeros((n + 2 * pad,) * 3)
    big[pad:pad + n, pad:pad + n, pad:pad + n] = f
    I, Iv = Q.shell_integrals(f, R, h, 6, aperiodic=True)
    Ib, Ivb = Q.shell_integrals(big, R, h, 6)
    s = (slice(pad, pad + n),) * 3
    assert np.max(np.abs(I - Ib[s])) < 1e-13
    assert np.max(np.abs(Iv - Ivb[(slice(None),) + s])) < 1e-13


def test_weighted_densities_uniform_fluid():
    rho = np.array([1.5, 0.4]).reshape(2, 1, 1, 1) * np.ones((2, 6, 6, 6))
    radii = [0.15, 0.27]
    w = Q.shell_weighted_densities(rho, radii, 0.1, 8)
    # bulk FMT values: n0 = sum rho, n1 = sum rho R, n2 = sum 4 pi R^2 rho, vectors 0
    assert np.allclose(w["n0"], 1.5 + 0.4, rtol=1e-12)
    assert np.allclose(w["n1"], 1.5 * 0.15 + 0.4 * 0.27, rtol=1e-12)
    assert np.allclose(w["n2"], 4 * math.pi * (1.5 * 0.15 ** 2 + 0.4 * 0.27 ** 2), rtol=1e-12)
    assert np.max(np.abs(w["n1v"])) < 1e-12 and np.max(np.abs(w["n2v"])) < 1e-12


def test_gaussian_delta_constant_field():
    n, h, R, alpha, c = 4, 0.05, 0.3, 0.1, 1.7
    f = np.full((n, n, n), c)
    I = Q.shell_integral_gaussian_delta(f, R, h, alpha)
    # int_R^3 delta_alpha(|x| - R) dx = 4 pi (R^2 + alpha^2 / 2), less a tail of order erfc(R / alpha)
    exact = 4.0 * math.pi * (R * R + 0.5 * alpha * alpha) * c
    assert np.max(np.abs(I - exact)) < 1e-4 * exact


@pytest.mark.parametrize("aperiodic", [False, True])
def test_pointwise_form_matches_whole_grid(aperiodic):
    rng = np.random.default_rng(7)
    shape, h, R = (6, 9, 5), 0.1, 0.33
    f = rng.random(shape)
    I, Iv = Q.shell_integrals(f, R, h, 6, aperiodic=aperiodic)
    pts = np.stack(np.meshgrid(*[np.arange(m) for m in shape], indexing="ij"), axis=-1).reshape(-1, 3)
    Ip, Ivp = Q.shell_integrals_at(f, R, h, 6, pts, aperiodic=aperiodic)
    assert np.max(np.abs(Ip - I.reshape(-1))) < 1e-13
    assert np.max(np.abs(Ivp - Iv.reshape(3, -1))) < 1e-13


def test_accuracy_ordering_against_closed_form():
    """Sec. 3.5 argues that the quadrature over spheres is more accurate than a
    Gaussian-smoothed delta with a volume rule; the spectral delta-shell weights
    of the main evaluation are exact for a field the grid resolves.  On a
    Gaussian bump (width 2 h) with the exact sphere integrals as reference:
    spectral < quadrature < smoothed delta (alpha = h and 2 h)."""
    import oracle
    import pnp_inputs as P
    n, L, s, R = 32, 4.8, 0.3, 0.25
    h = L / n
    x = h * np.arange(n)
    c = np.array([L / 2, L / 2 + 0.5 * h, L / 2 - 0.3 * h])
    X, Y, Z = np.meshgrid(x, x, x, indexing="ij")
    d = np.sqrt((X - c[0]) ** 2 + (Y - c[1]) ** 2 + (Z - c[2]) ** 2)
    f = np.exp(-d * d / (2 * s * s))
    I_ex, _ = Q.gaussian_bump_shell(d, R, s)
    scale = np.max(I_ex)
    prob = P.Problem(n=n, h=h, species=[P.Species(d=2 * R, q=0.0, rho_bulk=1.0, mu_el_bulk=0.0)], T=300.0,
                     terms=1, eps_r=16.6, sw_eps=None, sw_rout=None, sw_gamma=1.2, sw_prefactor=0.5,
                     precision=0, name="bump")
    e_spec = np.max(np.abs(oracle.weighted_densities(prob, f[None], "fft")["n2"] - I_ex)) / scale
    e_quad = np.max(np.abs(Q.shell_integrals(f, R, h, 8)[0] - I_ex)) / scale
    e_g1 = np.max(np.abs(Q.shell_integral_gaussian_delta(f, R, h, h) - I_ex)) / scale
    e_g2 = np.max(np.abs(Q.shell_integral_gaussian_delta(f, R, h, 2 * h) - I_ex)) / scale
    assert e_spec < 1e-9
    assert e_spec < e_quad < e_g1 < e_g2, (e_spec, e_quad, e_g1, e_g2)
