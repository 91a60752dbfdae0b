"""Stationary species (pnp_species.mobile = 0): a fixed site density (the
Gaussian sites of Sec. 2.3.2, coupled to the cations by a square well)
enters the weighted densities and pair terms like any species, but the
density updates leave it alone.

Checks, FP64 against the oracle (1e-10) and bit for bit where stated:
  * pnp_relax_densities: the stationary density is unchanged bit for bit,
    the mobile ones equal the oracle's update;
  * pnp_equilibrium: the same number of Picard steps as the oracle, the
    sites unchanged bit for bit, the converged ions self-consistent with
    the oracle's mu_ex computed with the sites present;
  * pool sessions and captured plans with a density update: the sites stay,
    the ions equal the batch call plus the relax entry point.
"""
import numpy as np
import pytest
import torch

import oracle
import pnp_inputs as P
from conftest import relerr, to_dev
from paper_1407_0674_amd import Pool
from test_oracle_equilibrium import electrolyte, sites

pytestmark = pytest.mark.gpu


def _with_sites(n=16, eps_site=0.05):
    prob, rho, bv = electrolyte(n, terms=P.TERMS_ALL)
    sp = list(prob.species) + [P.Species(0.2, 0.0, 0.0, 0.0, mobile=False)]
    eps = np.zeros((3, 3))
    eps[0, 2] = eps[2, 0] = eps_site
    prob = prob.with_(species=sp, sw_eps=eps, sw_rout=np.zeros((3, 3)))
    rs = sites(n, prob.h, [(0.4, 0.4, 0.4), (1.2, 1.0, 0.6)], 40.0, 1.0)
    rho = np.concatenate([rho, rs[None]])
    bv = np.concatenate([bv, np.zeros((1, n, n, n))])
    return prob, rho, bv


def test_relax_keeps_stationary_species(ev):
    prob, rho, _ = _with_sites()
    rng = np.random.default_rng(3)
    rho = rho * (1.0 + 0.2 * rng.uniform(-1, 1, size=rho.shape))
    rho[2] = sites(16, prob.h, [(0.4, 0.4, 0.4)], 40.0, 1.0)
    mu = rng.normal(size=rho.shape)
    mb = [0.3, -0.2, 0.7]
    rb = [s.rho_bulk for s in prob.species]
    ref = oracle.relax_densities(rho, mu, rb, mb, 0.3, clip=1.0, mobile=[True, True, False])
    rd = to_dev(rho)
    ev.relax(prob, rd, to_dev(mu), mb, lam=0.3, clip=1.0)
    got = rd.cpu().numpy()
    assert np.array_equal(got[2], rho[2])
    assert relerr(got[:2], ref[:2]) < 1e-14


@pytest.mark.parametrize("steps", [1, 5])
def test_equilibrium_steps_match_oracle(ev, steps):
    prob, rho, bv = _with_sites()
    ref, it_ref, res_ref = oracle.picard(prob, rho, beta_v=bv, lam=0.5, tol=0.0, max_iter=steps)
    rd = to_dev(rho)
    mu, it, res = ev.equilibrium(prob, rd, beta_v=to_dev(bv), lam=0.5, tol=0.0, max_iter=steps)
    got = rd.cpu().numpy()
    assert it == steps == it_ref
    assert np.array_equal(got[2], rho[2])
    assert relerr(got, ref) < 1e-10
    assert abs(res - res_ref) <= 1e-9 * max(1.0, res_ref)


def test_equilibrium_converges_with_sites(ev):
    prob, rho, bv = _with_sites()
    rd = to_dev(rho)
    _, it, res = ev.equilibrium(prob, rd, beta_v=to_dev(bv), lam=0.5, tol=1e-11, max_iter=400)
    assert res <= 1e-11
    out = rd.cpu().numpy()
    assert np.array_equal(out[2], rho[2])
    mu = oracle.mu_ex(prob, out, "fft")["total"]
    mb = oracle.bulk_mu_ex(prob)
    for i in range(2):
        rb = prob.species[i].rho_bulk
        assert np.max(np.abs(rb * np.exp(mb[i] - mu[i] - bv[i]) - out[i]) / rb) < 1e-9


def test_sessions_and_plans_keep_stationary_species(ev):
    prob, rho, _ = _with_sites()
    mb = oracle.bulk_mu_ex(prob)
    pool = Pool(ev, 1 << 28)
    sid = pool.open(prob, to_dev(rho), mu_bulk=list(mb), lam=0.3, clip=1.0)
    ref = to_dev(rho)
    for _ in range(3):
        assert pool.step([sid]) == [0]
        mus, _, st = ev.batch([prob], [ref])
        assert st == [0]
        ev.relax(prob, ref, mus[0], list(mb), lam=0.3, clip=1.0)
    r, m, s, steps = pool.view(sid)
    assert steps == 3
    assert torch.equal(r, ref)
    assert np.array_equal(r[2].cpu().numpy(), rho[2])
    assert not torch.equal(r[0], to_dev(rho)[0])
    # a captured plan with the density update does the same
    rp = to_dev(rho)
    plan = ev.plan([prob], [rp], relax=[(list(mb), 0.3, 1.0)])
    for _ in range(3):
        plan.launch()
    assert plan.status() == [0]
    assert torch.equal(rp, ref)
    del plan
    torch.cuda.synchronize()
    pool.close()
