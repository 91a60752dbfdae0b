"""GPU parity: the HIP path (through the C ABI) against the CPU FP64 oracle,
element by element on the same seeded inputs.

Tolerances (infinity-norm relative error per species and term):
FP64 path 1e-10, mixed FP32/FP64 path 1e-5.
"""
import math

import numpy as np
import pytest
import torch

import oracle
import pnp_inputs as P
from conftest import relerr, to_dev

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-10
MIXED_TOL = 1e-5


def _check_terms(res_gpu, ref, S, tol, terms):
    names = [("hs", P.TERM_HS), ("el", P.TERM_EC), ("sh", P.TERM_SW)]
    for k, (name, bit) in enumerate(names):
        for i in range(S):
            if terms & bit:
                assert relerr(res_gpu[k, i], ref[name][i]) < tol, (name, i, relerr(res_gpu[k, i], ref[name][i]))
            else:
                assert np.max(np.abs(res_gpu[k, i])) == 0.0


@pytest.mark.parametrize("route", ["direct"])
def test_config1_fp64_vs_direct_oracle(ev, route):
    prob, rho = P.config1()
    ref = oracle.mu_ex(prob, rho, route)
    mu, slot = ev.mu_ex(prob, to_dev(rho))
    mu, slot = mu.cpu().numpy(), slot.cpu().numpy()
    for i in range(prob.S):
        assert relerr(mu[i], ref["total"][i]) < FP64_TOL
        assert relerr(slot[i], ref["slotboom"][i]) < FP64_TOL
    mu3, _ = ev.mu_ex(prob, to_dev(rho), per_term=True)
    _check_terms(mu3.cpu().numpy(), ref, prob.S, FP64_TOL, prob.terms)


@pytest.mark.parametrize("n", [8, 16, 24, 32, 48])
def test_channel_fp64_per_term(ev, n):
    prob, rho = P.channel_problem(n, 1000 + n)
    ref = oracle.mu_ex(prob, rho, "fft")
    mu3, slot = ev.mu_ex(prob, to_dev(rho), per_term=True)
    _check_terms(mu3.cpu().numpy(), ref, prob.S, FP64_TOL, prob.terms)
    assert relerr(slot.cpu().numpy(), ref["slotboom"]) < FP64_TOL
    mu, _ = ev.mu_ex(prob, to_dev(rho))
    assert relerr(mu.cpu().numpy(), ref["total"]) < FP64_TOL


@pytest.mark.parametrize("n", [16, 24, 32])
def test_weighted_densities_fp64(ev, n):
    prob, rho = P.channel_problem(n, 2000 + n)
    ref = oracle.weighted_densities(prob, rho, "fft")
    nal = ev.weighted_densities(prob, to_dev(rho)).cpu().numpy()
    order = [ref["n0"], ref["n1"], ref["n2"], ref["n3"], *ref["n1v"], *ref["n2v"]]
    for k in range(10):
        scale = max(np.max(np.abs(order[k])), 1e-300)
        assert np.max(np.abs(nal[k] - order[k])) / scale < FP64_TOL, k


def test_weighted_densities_direct_oracle_config1(ev):
    prob, rho = P.config1()
    ref = oracle.weighted_densities(prob, rho, "direct")
    nal = ev.weighted_densities(prob, to_dev(rho)).cpu().numpy()
    order = [ref["n0"], ref["n1"], ref["n2"], ref["n3"], *ref["n1v"], *ref["n2v"]]
    for k in range(10):
        assert np.max(np.abs(nal[k] - order[k])) / np.max(np.abs(order[k])) < FP64_TOL, k


@pytest.mark.parametrize("terms", [P.TERM_HS, P.TERM_EC, P.TERM_SW, P.TERM_EC | P.TERM_SW, P.TERM_HS | P.TERM_SW])
def test_term_subsets_fp64(ev, terms):
    prob, rho = P.channel_problem(16, 3000 + terms)
    prob = prob.with_(terms=terms)
    ref = oracle.mu_ex(prob, rho, "fft")
    mu, slot = ev.mu_ex(prob, to_dev(rho))
    assert relerr(mu.cpu().numpy(), ref["total"]) < FP64_TOL
    assert relerr(slot.cpu().numpy(), ref["slotboom"]) < FP64_TOL


@pytest.mark.parametrize("n", [16, 32, 48])
def test_channel_mixed_per_term(ev, n):
    prob, rho = P.channel_problem(n, 4000 + n, precision=P.MIXED)
    ref = oracle.mu_ex(prob, rho, "fft")
    mu3, slot = ev.mu_ex(prob, to_dev(rho), per_term=True)
    _check_terms(mu3.cpu().numpy(), ref, prob.S, MIXED_TOL, prob.terms)


def test_config2_fp64_64(ev):
    prob, rho = P.config2()
    ref = oracle.mu_ex(prob, rho, "fft")
    mu3, slot = ev.mu_ex(prob, to_dev(rho), per_term=True)
    _check_terms(mu3.cpu().numpy(), ref, prob.S, FP64_TOL, prob.terms)
    assert relerr(slot.cpu().numpy(), ref["slotboom"]) < FP64_TOL


def test_high_packing_mixed_64(ev):
    prob, rho = P.config3(n=64)
    ref = oracle.mu_ex(prob, rho, "fft")
    mu3, slot = ev.mu_ex(prob, to_dev(rho), per_term=True)
    _check_terms(mu3.cpu().numpy(), ref, prob.S, MIXED_TOL, prob.terms)


def _py_single(eta):
    """beta mu_ex of a one-component hard-sphere fluid in the Percus-Yevick
    compressibility route, which the Rosenfeld functional reproduces in bulk."""
    return -math.log1p(-eta) + (14 * eta - 13 * eta ** 2 + 5 * eta ** 3) / (2 * (1 - eta) ** 3)


@pytest.mark.parametrize("eta", [1e-9, 1e-4, 0.0025, 0.2, 0.45, 0.6, 0.72])
def test_uniform_fluid_fp64_is_percus_yevick(ev, eta):
    # the packing fractions put 1 - n3 in every branch of the derivative
    # pass's logarithm: within 2^-9 of 1, just outside, and below 1/2
    d = 0.3
    rho_b = eta / (math.pi / 6 * d ** 3)
    prob = P.Problem(n=8, h=0.1, species=[P.Species(d, 0.0, rho_b)], T=300.0, terms=P.TERM_HS)
    rho = np.full(prob.shape, rho_b)
    mu, _ = ev.mu_ex(prob, to_dev(rho))
    got = mu.cpu().numpy()
    assert np.max(np.abs(got / _py_single(eta) - 1.0)) < 1e-12, eta
