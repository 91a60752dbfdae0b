"""Pins of the oracle's Picard equilibrium solve (the grand-ensemble state of
Sec. 3.2): a uniform bulk fluid is a fixed point; a very dilute hard-sphere
fluid in an external potential follows the Boltzmann law rho_b exp(-beta V);
a converged solution satisfies the equilibrium condition when mu_ex is
recomputed from it."""
import math

import numpy as np

import oracle
import pnp_inputs as P


def test_bulk_is_fixed_point():
    prob, _ = P.channel_problem(8, 11)
    prob = prob.with_(terms=P.TERM_HS | P.TERM_EC)
    rho = np.stack([np.full((8, 8, 8), s.rho_bulk) for s in prob.species])
    out, it, res = oracle.picard(prob, rho, lam=0.5, tol=1e-12)
    assert it == 1 and res < 1e-12
    assert np.max(np.abs(out - rho) / rho.max()) < 1e-12


def test_dilute_boltzmann_limit():
    # eta ~ 1e-9: mu_ex - mu_bulk is of order eta, so rho = rho_b exp(-beta V) to ~1e-8
    n, h, d = 16, 0.05, 0.3
    rb = 1e-9 / (math.pi / 6 * d ** 3)
    prob = P.Problem(n=n, h=h, species=[P.Species(d, 0.0, rb)], T=300.0, terms=P.TERM_HS)
    x = np.arange(n) * h
    bv = 0.8 * np.cos(2 * math.pi * x / (n * h))[:, None, None] * np.ones((1, n, n))
    bv = bv[None]
    out, it, res = oracle.picard(prob, np.full((1, n, n, n), rb), beta_v=bv, lam=1.0, tol=1e-13, max_iter=50)
    assert res <= 1e-13
    assert np.max(np.abs(out / (rb * np.exp(-bv)) - 1.0)) < 1e-7


def electrolyte(n=16, terms=P.TERM_HS | P.TERM_EC, eps_r=78.5):
    """1:1 electrolyte at 0.5 M (d = 0.30 / 0.35 nm) in water-like eps_r with a
    sinusoidal external potential of opposite sign for the two ions (plain
    Picard iteration converges here; with eps_r = 16.6 the MSA correlations are
    strong enough to drive it past close packing)."""
    sp = [P.Species(0.30, 1.0, 0.5 * P.MOLAR_TO_NM3), P.Species(0.35, -1.0, 0.5 * P.MOLAR_TO_NM3)]
    prob = P.Problem(n=n, h=0.1, species=sp, T=300.0, terms=terms, eps_r=eps_r)
    x = np.arange(n)
    bv = np.stack([sg * 0.6 * np.sin(2 * math.pi * x / n)[:, None, None] * np.ones((1, n, n)) for sg in (1.0, -1.0)])
    rho = np.stack([np.full((n, n, n), s.rho_bulk) for s in sp])
    return prob, rho, bv


def test_converged_state_is_self_consistent():
    prob, rho, bv = electrolyte()
    out, it, res = oracle.picard(prob, rho, beta_v=bv, lam=0.5, tol=1e-11, max_iter=300)
    assert res <= 1e-11
    mu = oracle.mu_ex(prob, out, "fft")["total"]
    mb = oracle.bulk_mu_ex(prob)
    rb = np.array([s.rho_bulk for s in prob.species])[:, None, None, None]
    target = rb * np.exp(mb[:, None, None, None] - mu - bv)
    assert np.max(np.abs(target - out) / rb) < 1e-10
    # cations gather where their potential is low, anions where theirs is
    assert out[0].reshape(16, -1).mean(axis=1).argmax() == bv[0].reshape(16, -1).mean(axis=1).argmin()


def sites(n, h, centres, alpha, rho0):
    """A stationary-site density of Gaussians, rho0 (alpha/pi)^(3/2) sum_k
    exp(-alpha |r - R_k|^2) with minimum-image distances (the site density
    form of Sec. 2.3.2)."""
    L = n * h
    c = np.arange(n) * h
    out = np.zeros((n, n, n))
    for R in centres:
        d = [c - R[a] - L * np.round((c - R[a]) / L) for a in range(3)]
        r2 = d[0][:, None, None] ** 2 + d[1][None, :, None] ** 2 + d[2][None, None, :] ** 2
        out += np.exp(-alpha * r2)
    return rho0 * (alpha / math.pi) ** 1.5 * out


def test_stationary_species_stay_and_mobile_ones_equilibrate():
    """A 1:1 electrolyte next to a stationary site density that attracts the
    cations by a square well: the sites keep their density bit for bit, the
    ions reach the equilibrium of mu_ex computed with the sites present, and
    the cations gather at the sites."""
    n, h = 16, 0.1
    prob, rho, bv = electrolyte(n, terms=P.TERMS_ALL)
    site = P.Species(0.2, 0.0, 0.0, 0.0, mobile=False)
    sp = list(prob.species) + [site]
    eps = np.zeros((3, 3))
    eps[0, 2] = eps[2, 0] = 0.05          # cation-site well [eV]
    rout = np.zeros((3, 3))
    prob = prob.with_(species=sp, sw_eps=eps, sw_rout=rout)
    rs = sites(n, h, [(0.4, 0.4, 0.4), (1.2, 1.0, 0.6)], 40.0, 1.0)
    rho = np.concatenate([rho, rs[None]])
    bv = np.concatenate([bv, np.zeros((1, n, n, n))])
    out, it, res = oracle.picard(prob, rho, beta_v=bv, lam=0.5, tol=1e-11, max_iter=400)
    assert res <= 1e-11
    assert np.array_equal(out[2], rs)
    mu = oracle.mu_ex(prob, out, "fft")["total"]
    mb = oracle.bulk_mu_ex(prob)
    for i in range(2):
        rb = prob.species[i].rho_bulk
        target = rb * np.exp(mb[i] - mu[i] - bv[i])
        assert np.max(np.abs(target - out[i]) / rb) < 1e-10
    # the well draws cations to the sites: more of them at a site centre than
    # with the well switched off
    off, _, res0 = oracle.picard(prob.with_(sw_eps=np.zeros((3, 3))), rho, beta_v=bv, lam=0.5, tol=1e-11,
                                 max_iter=400)
    assert res0 <= 1e-11 and np.array_equal(off[2], rs)
    assert out[0, 4, 4, 4] > 1.05 * off[0, 4, 4, 4]
