"""GPU free energies (pnp_free_energy) against the oracle's F_hs, F_el, F_sh
(Sec. 2.3), for every term subset, in FP64 (1e-10 relative to the larger of
|F| and 1) and mixed precision (1e-5); reductions run in a fixed order, so
repeated calls agree bit for bit; the returned per-term mu_ex is the
per-term evaluation's."""
import numpy as np
import pytest
import torch

import oracle
import pnp_inputs as P
from conftest import relerr, to_dev

pytestmark = pytest.mark.gpu


def _close(got, ref, tol):
    for k in ("hs", "el", "sh", "total"):
        assert abs(got[k] - ref[k]) <= tol * max(1.0, abs(ref[k])), (k, got[k], ref[k])


@pytest.mark.parametrize("terms", [P.TERM_HS, P.TERM_EC, P.TERM_SW, P.TERM_HS | P.TERM_SW, P.TERMS_ALL])
def test_free_energy_fp64(ev, terms):
    prob, rho = P.channel_problem(16, 4400 + terms)
    sp = [P.Species(s.d, s.q, s.rho_bulk, 0.2 * (i + 1)) for i, s in enumerate(prob.species)]
    prob = prob.with_(terms=terms, species=sp)
    ref = oracle.free_energy(prob, rho, "fft")
    got, mu3 = ev.free_energy(prob, to_dev(rho))
    _close(got, ref, 1e-10)
    mref = oracle.mu_ex(prob, rho, "fft")
    for k, name in enumerate(("hs", "el", "sh")):
        assert np.max(np.abs(mu3[k].cpu().numpy() - mref[name])) <= 1e-10 * max(1.0, np.max(np.abs(mref[name])))


@pytest.mark.parametrize("n", [24, 32, 48])
def test_free_energy_sizes_fp64(ev, n):
    prob, rho = P.channel_problem(n, 4500 + n)
    _close(ev.free_energy(prob, to_dev(rho))[0], oracle.free_energy(prob, rho, "fft"), 1e-10)


def test_free_energy_config1_and_mixed(ev):
    prob, rho = P.config1()
    _close(ev.free_energy(prob, to_dev(rho))[0], oracle.free_energy(prob, rho, "fft"), 1e-10)
    prob, rho = P.channel_problem(32, 4601, precision=P.MIXED)
    _close(ev.free_energy(prob, to_dev(rho))[0], oracle.free_energy(prob, rho, "fft"), 1e-5)


def test_free_energy_reproducible(ev):
    prob, rho = P.config3(n=64)
    rd = to_dev(rho)
    a = ev.free_energy(prob, rd)[0]
    b = ev.free_energy(prob, rd)[0]
    assert a == b


def test_free_energy_derivative_matches_mu(ev):
    """d F / d rho_i(r) = h^3 (beta mu_hs + beta mu_el + beta mu_sh / (2 c_sw) * ...):
    for HS and EC the functional derivative of F is h^3 beta mu (central
    differences at one grid point, FP64)."""
    prob, rho = P.channel_problem(16, 4700)
    prob = prob.with_(terms=P.TERM_HS | P.TERM_EC)
    h3 = prob.h ** 3
    _, mu3 = ev.free_energy(prob, to_dev(rho))
    mu = (mu3[0] + mu3[1]).cpu().numpy()
    for (i, x, y, z) in [(0, 3, 5, 7), (2, 11, 0, 9)]:
        eps = 1e-4 * rho[i, x, y, z]
        rp, rm = rho.copy(), rho.copy()
        rp[i, x, y, z] += eps
        rm[i, x, y, z] -= eps
        fd = (ev.free_energy(prob, to_dev(rp))[0]["total"] - ev.free_energy(prob, to_dev(rm))[0]["total"]) / (2 * eps * h3)
        assert abs(fd - mu[i, x, y, z]) < 1e-6 * max(1.0, abs(mu[i, x, y, z])), (fd, mu[i, x, y, z])
