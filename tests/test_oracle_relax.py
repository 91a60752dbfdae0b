"""Pins of the oracle's density update of the consumer stub (Sec. 3.2
relaxation toward the Boltzmann-like equilibrium of mu_ex)."""
import math

import numpy as np

import oracle
import pnp_inputs as P


def test_lambda_zero_is_identity():
    rng = np.random.default_rng(1)
    rho = rng.uniform(0.1, 2.0, size=(3, 4, 4, 4))
    mu = rng.normal(size=rho.shape)
    out = oracle.relax_densities(rho, mu, [1.0, 2.0, 3.0], [0.1, 0.2, 0.3], 0.0)
    assert np.array_equal(out, rho)


def test_lambda_one_is_equilibrium_density():
    # mu_ex above its bulk value by ln 2 halves the density; below by ln 3 triples it
    rho = np.full((2, 2, 2, 2), 7.0)
    mu = np.empty_like(rho)
    mu[0] = 0.4 + math.log(2.0)
    mu[1] = -0.1 - math.log(3.0)
    out = oracle.relax_densities(rho, mu, [1.5, 0.2], [0.4, -0.1], 1.0)
    assert np.allclose(out[0], 0.75, rtol=1e-15, atol=0)
    assert np.allclose(out[1], 0.6, rtol=1e-15, atol=0)


def test_bulk_state_is_fixed_point():
    # a uniform single-species fluid at its bulk density, with the bulk mu taken
    # from the Percus-Yevick closed form, stays put under any relaxation factor
    eta = 0.3
    d = 0.3
    rho_b = eta / (math.pi / 6.0 * d ** 3)
    mu_py = -math.log(1 - eta) + (14 * eta - 13 * eta ** 2 + 5 * eta ** 3) / (2 * (1 - eta) ** 3)
    sp = [P.Species(d=d, q=0.0, rho_bulk=rho_b)]
    prob = P.Problem(n=8, h=0.05, species=sp, T=300.0, terms=P.TERM_HS)
    rho = np.full((1, 8, 8, 8), rho_b)
    mu = oracle.mu_ex(prob, rho, "fft")["total"]
    assert abs(mu.max() - mu_py) < 1e-12 and abs(mu.min() - mu_py) < 1e-12
    for lam in (0.1, 0.5, 1.0):
        out = oracle.relax_densities(rho, mu, [rho_b], [mu_py], lam)
        assert np.max(np.abs(out - rho)) / rho_b < 1e-12


def test_limit_bounds_the_exponent():
    # with a limit c the target density lies in [rho_b e^-c, rho_b e^c]
    rho = np.full((1, 2, 2, 2), 3.0)
    mu = np.array([[[[-50.0, 0.2], [50.0, -0.1]], [[0.0, 7.0], [-7.0, 0.5]]]])
    out = oracle.relax_densities(rho, mu, [2.0], [0.0], 1.0, clip=0.5)
    g = np.clip(-mu, -0.5, 0.5)
    assert np.allclose(out, 2.0 * np.exp(g), rtol=1e-15, atol=0)
    assert out.max() <= 2.0 * math.exp(0.5) * (1 + 1e-15) and out.min() >= 2.0 * math.exp(-0.5) * (1 - 1e-15)
    # clip <= 0: no limit
    out0 = oracle.relax_densities(rho, mu, [2.0], [0.0], 1.0, clip=0.0)
    assert np.allclose(out0, 2.0 * np.exp(-mu), rtol=1e-15, atol=0)


def test_stationary_species_keep_their_density():
    # a stationary species (mobile = False) is left as it is, bit for bit; the
    # mobile ones get exactly the update they get when every species moves
    rng = np.random.default_rng(5)
    rho = rng.uniform(0.1, 2.0, size=(3, 4, 4, 4))
    mu = rng.normal(size=rho.shape)
    args = (rho, mu, [1.0, 2.0, 3.0], [0.1, 0.2, 0.3], 0.4)
    all_mobile = oracle.relax_densities(*args, clip=0.7)
    out = oracle.relax_densities(*args, clip=0.7, mobile=[True, False, True])
    assert np.array_equal(out[1], rho[1])
    assert np.array_equal(out[[0, 2]], all_mobile[[0, 2]])
    assert not np.array_equal(all_mobile[1], rho[1])
