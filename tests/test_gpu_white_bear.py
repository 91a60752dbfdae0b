"""GPU parity of the modified (White Bear) hard-sphere functional of
Sec. 2.3.1 (PNP_TERM_HS_WB) against the oracle: per term, in FP64 (1e-10)
and mixed precision (1e-5), on channel electrolytes whose packing fraction
crosses the switch between the series and the closed form of phi3 (0.05),
at high packing, in free energies, in batches that mix both functionals,
and against the Carnahan-Starling value of a uniform fluid."""
import math

import numpy as np
import pytest
import torch

import oracle
import pnp_inputs as P
from conftest import relerr, to_dev

pytestmark = pytest.mark.gpu

WB_ALL = P.TERM_HS_WB | P.TERM_EC | P.TERM_SW


def _per_term(ev, prob, rho, tol):
    ref = oracle.mu_ex(prob, rho, "fft")
    mu3, slot = ev.mu_ex(prob, to_dev(rho), per_term=True)
    mu3 = mu3.cpu().numpy()
    for k, name in enumerate(("hs", "el", "sh")):
        for i in range(prob.S):
            assert relerr(mu3[k, i], ref[name][i]) < tol, (name, i, relerr(mu3[k, i], ref[name][i]))
    # exp(-mu) carries the absolute error of mu as a relative one
    assert relerr(slot.cpu().numpy(), ref["slotboom"]) < tol * max(1.0, float(np.max(np.abs(ref["total"]))))
    mu, _ = ev.mu_ex(prob, to_dev(rho))
    assert relerr(mu.cpu().numpy(), ref["total"]) < tol
    return ref


@pytest.mark.parametrize("n", [16, 24, 32])
def test_wb_channel_fp64(ev, n):
    prob, rho = P.channel_problem(n, 5100 + n, terms=WB_ALL)
    ref = _per_term(ev, prob, rho, 1e-10)
    n3 = ref["n"]["n3"]
    assert n3.min() < 0.05 < n3.max()  # both forms of phi3 are exercised


def test_wb_differs_from_rosenfeld(ev):
    prob, rho = P.channel_problem(16, 5200, terms=WB_ALL)
    a = ev.mu_ex(prob, to_dev(rho))[0].cpu().numpy()
    b = ev.mu_ex(prob.with_(terms=P.TERMS_ALL), to_dev(rho))[0].cpu().numpy()
    assert np.max(np.abs(a - b)) > 1e-4


@pytest.mark.parametrize("n", [32, 48])
def test_wb_channel_mixed(ev, n):
    prob, rho = P.channel_problem(n, 5300 + n, precision=P.MIXED, terms=WB_ALL)
    _per_term(ev, prob, rho, 1e-5)


def test_wb_high_packing(ev):
    prob, rho = P.config3(n=64)
    prob = prob.with_(terms=WB_ALL, precision=P.FP64)
    _per_term(ev, prob, rho, 1e-10)
    _per_term(ev, prob.with_(precision=P.MIXED), rho, 1e-5)


@pytest.mark.parametrize("eta", [0.03, 0.3, 0.45])
def test_wb_uniform_fluid_is_carnahan_starling(ev, eta):
    d = 0.3
    sp = [P.Species(d, 0.0, eta / (math.pi / 6.0 * d ** 3))]
    prob = P.Problem(n=16, h=0.05, species=sp, T=300.0, terms=P.TERM_HS_WB)
    rho = np.full((1, 16, 16, 16), sp[0].rho_bulk)
    cs = (8 * eta - 9 * eta ** 2 + 3 * eta ** 3) / (1 - eta) ** 3
    mu = ev.mu_ex(prob, to_dev(rho))[0].cpu().numpy()
    assert np.max(np.abs(mu - cs)) < 1e-12 * cs
    mu = ev.mu_ex(prob.with_(precision=P.MIXED), to_dev(rho))[0].cpu().numpy()
    assert np.max(np.abs(mu - cs)) < 1e-5 * cs


def test_wb_free_energy(ev):
    prob, rho = P.channel_problem(24, 5400, terms=WB_ALL)
    ref = oracle.free_energy(prob, rho, "fft")
    got, _ = ev.free_energy(prob, to_dev(rho))
    for k in ("hs", "el", "sh", "total"):
        assert abs(got[k] - ref[k]) <= 1e-10 * max(1.0, abs(ref[k])), (k, got[k], ref[k])


def test_wb_batch_mixes_functionals(ev):
    """One batch holding Rosenfeld and White Bear instances of one size: each
    result equals its own single call bit for bit."""
    probs, rhos = [], []
    for k, terms in enumerate((WB_ALL, P.TERMS_ALL, P.TERM_HS_WB, P.TERM_HS)):
        prob, rho = P.channel_problem(32, 5500 + k, terms=terms)
        probs.append(prob)
        rhos.append(to_dev(rho))
    mus, slots, st = ev.batch(probs, rhos)
    assert st == [0] * len(probs)
    for prob, rd, mu, sl in zip(probs, rhos, mus, slots):
        m1, s1 = ev.mu_ex(prob, rd)
        assert torch.equal(mu, m1), prob.terms
        assert torch.equal(sl, s1), prob.terms


def test_wb_uniform_mixture_is_bmcsl(ev):
    from test_oracle_fmt import bmcsl_mu
    ds, rb = (0.15, 0.3, 0.4), (3.0, 2.0, 4.0)
    prob = P.Problem(n=16, h=0.05, species=[P.Species(ds[i], 0.0, rb[i]) for i in range(3)], T=300.0,
                     terms=P.TERM_HS_WB)
    rho = np.stack([np.full((16, 16, 16), r) for r in rb])
    mu = ev.mu_ex(prob, to_dev(rho))[0].cpu().numpy()
    ref = bmcsl_mu(ds, rb)
    for i in range(3):
        assert np.max(np.abs(mu[i] - ref[i])) < 1e-12 * np.max(np.abs(ref))
