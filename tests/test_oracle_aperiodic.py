"""Pins of the oracle's aperiodic (zero-extension) mode (Sec. 3.4, Sec. 3.5).

* the 1D construction of Sec. 3.4 (two length-2N circular convolutions, one
  with a reflected kernel) equals the trapezoidal sum written out, with the
  reflected index g_(N-1-i); the printed g_(N-2-i) does not;
* the square-well and electrostatic-correlation terms equal the finite sums
  over the domain with the kernels of the doubled grid, written out point by
  point (no FFT);
* the hard-sphere term through numpy's FFT equals the oracle's direct route
  (explicit kernels and O(N^2) sums) on the doubled grid;
* the hard-sphere term equals its sums over the domain written out point by
  point: weighted densities at the domain points from the domain's
  densities, then the back-convolution of the derivative fields over the
  domain only (Sec. 2.3.1 integrates Phi_hs over Omega);
* central differences of F_hs = h^3 sum_Omega Phi_hs against single-point
  density changes give h^3 beta mu_hs, at faces, edges, corners and inside;
* the mode differs from the periodic one and is mirror-covariant about the
  domain's centre (x -> n - 1 - x).
"""
import itertools

import numpy as np
import pytest

import oracle
import pnp_inputs as P
from oracle.aperiodic import (extend, linear_convolution_1d, mu_ex_aperiodic,
                              split_convolution_1d)
from oracle.discrete import build_operator, real_space_kernel


@pytest.mark.parametrize("N", [1, 2, 3, 5, 8, 13])
def test_split_1d_equals_trapezoidal_sum(N):
    rng = np.random.default_rng(100 + N)
    f, g = rng.normal(size=N), rng.normal(size=N)
    ref = linear_convolution_1d(f, g)
    assert np.max(np.abs(split_convolution_1d(f, g, shift=1) - ref)) < 1e-13
    if N >= 2:  # the printed reflected index misses the second sum by one place
        assert np.max(np.abs(split_convolution_1d(f, g, shift=2) - ref)) > 1e-3


def test_linear_sum_1d_brute_force_small():
    f = np.array([1.0, 2.0, 3.0])
    g = np.array([10.0, 1.0, 0.1])
    # h_0 = 1*10 + 2*1 + 3*0.1, h_1 = 1*1 + 2*10 + 3*1, h_2 = 1*0.1 + 2*1 + 3*10
    assert np.allclose(linear_convolution_1d(f, g), [12.3, 24.0, 32.1], rtol=0, atol=1e-12)


def _small_problem(n, seed, terms):
    rng = np.random.default_rng(seed)
    sp = [P.Species(0.30, +1.0, 0.9), P.Species(0.40, -1.0, 0.9)]
    eps, rout = P.uniform_well(sp, 0.2, 0.15)
    prob = P.Problem(n=n, h=0.1, species=sp, T=300.0, terms=terms, sw_eps=eps, sw_rout=rout)
    rho = P.uniform_noise(rng, n, [s.rho_bulk for s in sp], 0.4)
    return prob, rho


def _domain_sum(K, field, n):
    """out[r] = h^3-free sum over r' in the n^3 domain of K[(r - r') mod 2n] field[r']."""
    n2 = K.shape[0]
    out = np.zeros((n, n, n))
    idx = np.arange(n)
    for (x, y, z) in itertools.product(range(n), repeat=3):
        dx = (x - idx) % n2
        dy = (y - idx) % n2
        dz = (z - idx) % n2
        out[x, y, z] = np.sum(K[np.ix_(dx, dy, dz)] * field)
    return out


@pytest.mark.parametrize("term", [P.TERM_SW, P.TERM_EC])
def test_linear_terms_are_domain_sums(term):
    n = 5
    prob, rho = _small_problem(n, 7 + term, term)
    got = mu_ex_aperiodic(prob, rho, "fft")
    op = build_operator(prob.with_(n=2 * n), half=False)
    h3 = prob.h ** 3
    rb = np.array([s.rho_bulk for s in prob.species])
    for i in range(2):
        ref = np.zeros((n, n, n))
        for j in range(2):
            if term == P.TERM_SW:
                K = real_space_kernel(op.u_hat[i][j].astype(complex), 2 * n, prob.h)
                ref += op.c_sw * op.beta * h3 * _domain_sum(K, rho[j], n)
            else:
                K = real_space_kernel(op.C_hat[i][j].astype(complex), 2 * n, prob.h)
                ref -= h3 * _domain_sum(K, rho[j] - rb[j], n)
        key = "sh" if term == P.TERM_SW else "el"
        if term == P.TERM_EC:
            ref += prob.species[i].mu_el_bulk
        assert np.max(np.abs(got[key][i] - ref)) < 1e-11 * max(1.0, np.max(np.abs(ref))), (key, i)


def test_hard_spheres_fft_equals_direct_route():
    n = 4
    prob, rho = _small_problem(n, 11, P.TERM_HS)
    a = mu_ex_aperiodic(prob, rho, "fft")
    b = mu_ex_aperiodic(prob, rho, "direct")
    assert np.max(np.abs(a["hs"] - b["hs"])) < 1e-11 * np.max(np.abs(b["hs"]))
    # weighted densities reach outside the domain (spheres that stick out)
    assert np.max(np.abs(a["n_ext"]["n3"][n:, :, :])) > 1e-3


def _hs_kernels(op, n2, h, i):
    """Real-space kernels of species i on the doubled grid: the four scalar
    weights, then the three components of the two vector weights
    (-i khat V, the outward shell), in the order n0..n3, n1v, n2v."""
    w = op.w[i]
    ks = [real_space_kernel(w[a].astype(complex), n2, h) for a in ("w0", "w1", "w2", "w3")]
    for v in ("v1", "v2"):
        ks += [real_space_kernel(-1j * op.khat[c] * w[v], n2, h) for c in range(3)]
    return ks


def _domain_correlation(K, field, n):
    """out[r] = sum over r' in the n^3 domain of K[(r' - r) mod 2n] field[r'], r in the domain."""
    n2 = K.shape[0]
    out = np.zeros((n, n, n))
    idx = np.arange(n)
    for (x, y, z) in itertools.product(range(n), repeat=3):
        out[x, y, z] = np.sum(K[np.ix_((idx - x) % n2, (idx - y) % n2, (idx - z) % n2)] * field)
    return out


@pytest.mark.parametrize("terms", [P.TERM_HS, P.TERM_HS_WB])
def test_hard_sphere_term_is_domain_sum(terms):
    n = 4
    prob, rho = _small_problem(n, 17 + terms, terms)
    got = mu_ex_aperiodic(prob, rho, "fft")["hs"]
    op = build_operator(prob.with_(n=2 * n), half=False)
    h3 = prob.h ** 3
    kers = [_hs_kernels(op, 2 * n, prob.h, i) for i in range(2)]
    # weighted densities at the domain points (correlation over the domain)
    nal = [sum(h3 * _domain_correlation(kers[i][a], rho[i], n) for i in range(2)) for a in range(10)]
    dfn = oracle.dphi_hs_wb if terms == P.TERM_HS_WB else oracle.dphi_hs
    d = dfn(nal[0], nal[1], nal[2], nal[3], np.stack(nal[4:7]), np.stack(nal[7:10]))
    dl = [d["d0"], d["d1"], d["d2"], d["d3"], *d["d1v"], *d["d2v"]]
    for i in range(2):
        # back-convolution over the domain: sum_r' dPhi_a[r'] K_a[r - r']
        ref = sum(h3 * _domain_sum(kers[i][a], dl[a], n) for a in range(10))
        assert np.max(np.abs(got[i] - ref)) < 1e-11 * np.max(np.abs(ref)), i


def _f_hs_domain(prob, rho, n):
    """F_hs = h^3 sum over the domain of Phi_hs of the zero-extended densities."""
    big = prob.with_(n=2 * n)
    nal = oracle.weighted_densities(big, extend(rho, 2 * n), "fft")
    phi = (oracle.phi_hs_wb if prob.terms & P.TERM_HS_WB else oracle.phi_hs)(
        nal["n0"], nal["n1"], nal["n2"], nal["n3"], nal["n1v"], nal["n2v"])
    return prob.h ** 3 * float(np.sum(phi[:n, :n, :n]))


@pytest.mark.parametrize("terms", [P.TERM_HS, P.TERM_HS_WB])
def test_hard_sphere_term_is_derivative_of_domain_free_energy(terms):
    n = 6
    prob, rho = _small_problem(n, 29 + terms, terms)
    mu = mu_ex_aperiodic(prob, rho, "fft")["hs"]
    h3 = prob.h ** 3
    scale = float(np.max(np.abs(mu)))
    for (i, x, y, z) in [(0, 0, 0, 0), (1, n - 1, 0, 2), (0, 2, n - 1, n - 1), (1, 3, 2, 0), (0, 2, 3, 3),
                         (1, n - 1, n - 1, n - 1)]:
        step = 1e-4 * rho[i, x, y, z]
        rp, rm = rho.copy(), rho.copy()
        rp[i, x, y, z] += step
        rm[i, x, y, z] -= step
        fd = (_f_hs_domain(prob, rp, n) - _f_hs_domain(prob, rm, n)) / (2.0 * step * h3)
        assert abs(fd - mu[i, x, y, z]) < 2e-7 * scale, (i, x, y, z, fd, mu[i, x, y, z])


def test_differs_from_periodic_and_mirror_covariant():
    n = 6
    prob, rho = _small_problem(n, 13, P.TERMS_ALL)
    ap = mu_ex_aperiodic(prob, rho, "fft")
    per = oracle.mu_ex(prob, rho, "fft")
    assert np.max(np.abs(ap["total"] - per["total"])) > 1e-2
    flip = mu_ex_aperiodic(prob, rho[:, ::-1, :, :].copy(), "fft")
    assert np.max(np.abs(flip["total"] - ap["total"][:, ::-1, :, :])) < 1e-11 * np.max(np.abs(ap["total"]))


def test_extend_places_domain_at_corner():
    x = np.arange(8.0).reshape(1, 2, 2, 2)
    e = extend(x, 4)
    assert e.shape == (1, 4, 4, 4)
    assert np.array_equal(e[:, :2, :2, :2], x) and e.sum() == x.sum()
