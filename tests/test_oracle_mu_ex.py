"""Pins for the assembled beta*mu_ex: bulk closed forms (scaled-particle /
Percus-Yevick, the square-well integral, the MSA k = 0 integral), functional
derivative consistency with the free energies, symmetries, and the local
density limit of vanishing radii."""
import math

import numpy as np
import pytest

import oracle
import pnp_inputs as P
from conftest import relerr
from test_oracle_fmt import spt_mu

M = P.MOLAR_TO_NM3


def _uniform(prob, rho_b):
    n = prob.n
    return np.broadcast_to(np.asarray(rho_b)[:, None, None, None], (len(rho_b), n, n, n)).copy()


def test_config1_bulk_values():
    prob, _ = P.config1()
    rho = _uniform(prob, [M, M])
    r = oracle.mu_ex(prob, rho, "fft")
    assert np.allclose(r["hs"], spt_mu([M, M], [0.3, 0.3])[0], rtol=1e-12, atol=0)
    assert np.allclose(r["hs"], 0.14069489802580665, rtol=1e-12, atol=0)
    # square well: c_sw beta sum_j rho_j (-eps) (4 pi/3)(r_out^3 - sigma^3)
    b = 1.0 / (1.380649e-23 / 1.602176634e-19 * 300.0)
    exp_sh = 0.5 * b * 2 * M * (-0.3) * 4 * math.pi / 3 * (0.6 ** 3 - 0.3 ** 3)
    assert np.allclose(r["sh"], exp_sh, rtol=1e-12, atol=0)
    # the same number evaluated with k_B rounded to 10 digits
    assert exp_sh == pytest.approx(-5.5325892291873515, rel=1e-9)


def test_three_species_bulk_hs():
    sp = [P.Species(d, 1.0, M) for d in (0.15, 0.30, 0.40)]
    prob = P.Problem(n=8, h=0.05, species=sp, T=300.0, terms=P.TERM_HS)
    r = oracle.mu_ex(prob, _uniform(prob, [M, M, M]), "fft")
    exp = spt_mu([M, M, M], [0.15, 0.30, 0.40])
    for i in range(3):
        assert np.allclose(r["hs"][i], exp[i], rtol=1e-12, atol=0)
    assert exp == pytest.approx([0.0930474206, 0.2160371203, 0.3419525990], rel=1e-9)


def _msa_C0(qi, qj, lB, kappa, sigma):
    xi = kappa * sigma
    B = (xi + 1.0 - math.sqrt(1.0 + 2.0 * xi)) / xi          # as printed, Sec. 2.3.4
    # int C(r) d^3r over r <= sigma of -qi qj lB [2B/s - (B/s)^2 r - 1/r]
    return -qi * qj * lB * math.pi * sigma ** 2 * (8.0 * B / 3.0 - B * B - 2.0)


def test_ec_uniform_offset():
    prob, _ = P.config2(n=8)
    prob = prob.with_(terms=P.TERM_EC,
                      species=[P.Species(s.d, s.q, s.rho_bulk, mu_el_bulk=0.1 * i)
                               for i, s in enumerate(prob.species)])
    rb = np.array([s.rho_bulk for s in prob.species])
    delta = np.array([0.05, -0.02, 0.01])
    r = oracle.mu_ex(prob, _uniform(prob, rb + delta), "fft")
    lB = oracle.bjerrum_length(prob.T, prob.eps_r)
    kappa = math.sqrt(oracle.kappa_squared(prob.T, prob.eps_r, rb, [s.q for s in prob.species]))
    for i, si in enumerate(prob.species):
        exp = si.mu_el_bulk - sum(delta[j] * _msa_C0(si.q, sj.q, lB, kappa, 0.5 * (si.d + sj.d))
                                  for j, sj in enumerate(prob.species))
        assert np.allclose(r["el"][i], exp, rtol=1e-11, atol=1e-13)


def test_ec_c0_config1_pair():
    lB = oracle.bjerrum_length(300.0, 16.6)
    kappa = math.sqrt(oracle.kappa_squared(300.0, 16.6, [M, M], [1.0, -1.0]))
    # reference value computed with e^2/(4 pi eps0) = 1.439964547 eV nm (10 digits)
    assert _msa_C0(1.0, 1.0, lB, kappa, 0.3) == pytest.approx(1.0490540718075125, rel=1e-8)


@pytest.mark.parametrize("term,factor", [(P.TERM_HS, 1.0), (P.TERM_EC, 1.0), (P.TERM_SW, 2.0)])
def test_functional_derivative_consistency(term, factor):
    """mu_i[s] = h^-3 dF/drho_i[s]; the square-well chemical potential carries
    the printed 1/2, so there dF/drho = 2 mu_sh."""
    prob, rho = P.channel_problem(8, 21)
    prob = prob.with_(terms=term)
    r = oracle.mu_ex(prob, rho, "fft")
    key = {P.TERM_HS: "hs", P.TERM_EC: "el", P.TERM_SW: "sh"}[term]
    h3 = prob.h ** 3
    for (i, x, y, z) in [(0, 1, 2, 3), (2, 7, 0, 5), (1, 4, 4, 4)]:
        eps = 1e-4 * rho[i, x, y, z]
        rp, rm = rho.copy(), rho.copy()
        rp[i, x, y, z] += eps
        rm[i, x, y, z] -= eps
        fd = (oracle.free_energy(prob, rp)["total"] - oracle.free_energy(prob, rm)["total"]) / (2 * eps * h3)
        assert fd == pytest.approx(factor * r[key][i, x, y, z], rel=2e-7, abs=1e-9)


def _perm_prob(prob, perm):
    sp = [prob.species[p] for p in perm]
    eps = prob.sw_eps[np.ix_(perm, perm)]
    rout = prob.sw_rout[np.ix_(perm, perm)]
    return prob.with_(species=sp, sw_eps=eps, sw_rout=rout)


def test_symmetries():
    prob, rho = P.channel_problem(12, 31)
    base = oracle.mu_ex(prob, rho, "fft")["total"]
    # translation by a grid vector
    sh = (1, 5, 7)
    t = oracle.mu_ex(prob, np.roll(rho, sh, axis=(1, 2, 3)), "fft")["total"]
    assert relerr(t, np.roll(base, sh, axis=(1, 2, 3))) < 1e-13
    # species permutation
    perm = [2, 0, 1]
    p = oracle.mu_ex(_perm_prob(prob, perm), rho[perm], "fft")["total"]
    assert relerr(p, base[perm]) < 1e-13
    # mirror x -> -x
    mir = lambda a: np.roll(a[:, ::-1], 1, axis=1)
    m = oracle.mu_ex(prob, mir(rho), "fft")["total"]
    assert relerr(m, mir(base)) < 1e-13
    # 90 degree rotation (swap x and z)
    rot = lambda a: np.transpose(a, (0, 3, 2, 1))
    q = oracle.mu_ex(prob, rot(rho), "fft")["total"]
    assert relerr(q, rot(base)) < 1e-13


def test_charge_reversal_leaves_ec_unchanged():
    prob, rho = P.channel_problem(8, 41)
    prob = prob.with_(terms=P.TERM_EC)
    a = oracle.mu_ex(prob, rho, "fft")["el"]
    flip = prob.with_(species=[P.Species(s.d, -s.q, s.rho_bulk) for s in prob.species])
    b = oracle.mu_ex(flip, rho, "fft")["el"]
    assert relerr(b, a) < 1e-14


def test_vanishing_radius_is_local_density_limit():
    # the paper's electron has d = 0.001 nm on grids of ~0.05 nm: the FMT term
    # tends to the bulk formula at the local density
    n = 8
    sp = [P.Species(0.002, -1.0, 50.0), P.Species(0.001, 1.0, 80.0)]
    prob = P.Problem(n=n, h=0.05, species=sp, T=300.0, terms=P.TERM_HS)
    rng = np.random.default_rng(2)
    rho = np.stack([50.0 * (1 + 0.3 * rng.uniform(-1, 1, (n, n, n))),
                    80.0 * (1 + 0.3 * rng.uniform(-1, 1, (n, n, n)))])
    r = oracle.mu_ex(prob, rho, "fft")["hs"]
    for pt in [(1, 2, 3), (5, 5, 0)]:
        loc = spt_mu([rho[0][pt], rho[1][pt]], [0.002, 0.001])
        for i in range(2):
            assert r[i][pt] == pytest.approx(loc[i], rel=2e-3)


def test_slotboom_is_exp_of_minus_total():
    prob, rho = P.config1()
    r = oracle.mu_ex(prob, rho, "fft")
    assert np.allclose(r["slotboom"], np.exp(-r["total"]), rtol=1e-15)
