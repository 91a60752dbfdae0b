"""GPU edge cases against the oracle and exact properties: one and up to
eight species (the back pass then switches to output chunks of four), in
both precisions; the degenerate inputs of the method (all densities zero,
uniform bulk densities, a single point of density); the largest grid with
the largest species count, checked by a property that holds at any size
(uniform bulk densities give the bulk chemical potential everywhere)."""
import numpy as np
import pytest
import torch

import oracle
import pnp_inputs as P
from conftest import relerr, to_dev
from paper_1407_0674_amd import bulk_mu_ex

pytestmark = pytest.mark.gpu


def _per_term(ev, prob, rho, tol):
    ref = oracle.mu_ex(prob, rho, "fft")
    mu3, _ = ev.mu_ex(prob, to_dev(rho), per_term=True)
    mu3 = mu3.cpu().numpy()
    for k, name in enumerate(("hs", "el", "sh")):
        for i in range(prob.S):
            assert relerr(mu3[k, i], ref[name][i]) < tol, (prob.S, name, i, relerr(mu3[k, i], ref[name][i]))
    mu, slot = ev.mu_ex(prob, to_dev(rho))
    assert relerr(mu.cpu().numpy(), ref["total"]) < tol
    return ref


@pytest.mark.parametrize("S", [1, 5, 6, 8])
def test_species_counts_fp64(ev, S):
    prob, rho = P.many_species(16, S, 8000 + S)
    _per_term(ev, prob, rho, 1e-10)


@pytest.mark.parametrize("S", [1, 5, 8])
def test_species_counts_mixed(ev, S):
    prob, rho = P.many_species(24, S, 8100 + S, precision=P.MIXED)
    _per_term(ev, prob, rho, 1e-5)


def test_eight_species_batch_equals_alone(ev):
    probs, rhos = [], []
    for k, S in enumerate((8, 3, 6)):
        p, r = P.many_species(16, S, 8200 + k, precision=P.MIXED)
        probs.append(p)
        rhos.append(to_dev(r))
    mus, slots, st = ev.batch(probs, rhos)
    assert st == [0, 0, 0]
    for p, rd, mu, sl in zip(probs, rhos, mus, slots):
        m1, s1 = ev.mu_ex(p, rd)
        assert torch.equal(mu, m1) and torch.equal(sl, s1)


def test_zero_densities(ev):
    prob, rho = P.channel_problem(16, 8300)
    z = np.zeros_like(rho)
    ref = _per_term(ev, prob, z, 1e-10)
    assert np.max(np.abs(ref["hs"])) == 0.0  # no hard-sphere contribution without particles


def test_single_point_density(ev):
    prob, _ = P.channel_problem(16, 8301)
    rho = np.zeros((prob.S, 16, 16, 16))
    rho[1, 3, 7, 11] = 5.0
    _per_term(ev, prob, rho, 1e-10)


@pytest.mark.parametrize("precision,tol", [(P.FP64, 1e-10), (P.MIXED, 1e-5)])
def test_uniform_bulk_is_bulk_value(ev, precision, tol):
    prob, _ = P.channel_problem(32, 8302, precision=precision)
    sp = [P.Species(s.d, s.q, s.rho_bulk, 0.3 * (i - 1)) for i, s in enumerate(prob.species)]
    prob = prob.with_(species=sp)
    rho = np.stack([np.full((32, 32, 32), s.rho_bulk) for s in sp])
    mu = ev.mu_ex(prob, to_dev(rho))[0].cpu().numpy()
    mb = bulk_mu_ex(prob)
    for i in range(prob.S):
        assert np.max(np.abs(mu[i] - mb[i])) < tol * max(1.0, abs(mb[i])), i


def test_largest_grid_eight_species(ev):
    """256^3 with S = 8 in mixed precision (the chunked back pass at full
    size): uniform bulk densities give the bulk value at every point."""
    prob, _ = P.many_species(256, 8, 8400, precision=P.MIXED)
    rb = torch.tensor([s.rho_bulk for s in prob.species], dtype=torch.float64, device="cuda:0")
    rho = rb[:, None, None, None].expand(8, 256, 256, 256).contiguous()
    mu, slot = ev.mu_ex(prob, rho)
    mb = torch.tensor(bulk_mu_ex(prob), dtype=torch.float64, device="cuda:0")
    err = (mu - mb[:, None, None, None]).abs().amax().item()
    assert err < 1e-5 * max(1.0, mb.abs().max().item()), err
    assert torch.isfinite(slot).all()
    del rho, mu, slot
    torch.cuda.empty_cache()
