"""Pins for the FMT derivatives: finite differences of the printed Phi_hs,
and the bulk Percus-Yevick / scaled-particle closed forms."""
import math

import numpy as np
import pytest

from oracle import dphi_hs, phi_hs


def _point(rng):
    n3 = rng.uniform(0.05, 0.6)
    return dict(n0=rng.uniform(1, 10), n1=rng.uniform(0.1, 2), n2=rng.uniform(1, 8), n3=n3,
                n1v=rng.uniform(-0.5, 0.5, size=3), n2v=rng.uniform(-2, 2, size=3))


@pytest.mark.parametrize("seed", range(5))
def test_derivatives_match_finite_differences(seed):
    rng = np.random.default_rng(seed)
    p = _point(rng)
    args = lambda q: (np.array(q["n0"]), np.array(q["n1"]), np.array(q["n2"]), np.array(q["n3"]),
                      np.asarray(q["n1v"])[:, None], np.asarray(q["n2v"])[:, None])
    d = dphi_hs(*args(p))
    for key, dk in (("n0", "d0"), ("n1", "d1"), ("n2", "d2"), ("n3", "d3")):
        eps = 1e-6 * max(1.0, abs(p[key]))
        qp, qm = dict(p), dict(p)
        qp[key] = p[key] + eps
        qm[key] = p[key] - eps
        fd = (phi_hs(*args(qp)) - phi_hs(*args(qm))) / (2 * eps)
        assert float(d[dk]) == pytest.approx(float(fd), rel=1e-7, abs=1e-8), key
    for key, dk in (("n1v", "d1v"), ("n2v", "d2v")):
        for c in range(3):
            eps = 1e-6
            qp, qm = dict(p), dict(p)
            qp[key] = np.array(p[key]); qp[key][c] += eps
            qm[key] = np.array(p[key]); qm[key][c] -= eps
            fd = (phi_hs(*args(qp)) - phi_hs(*args(qm))) / (2 * eps)
            assert float(d[dk][c]) == pytest.approx(float(fd), rel=1e-7, abs=1e-8), (key, c)


def _bulk_mu(rho, d):
    """beta mu_i from the FMT derivatives at bulk weighted densities."""
    R = 0.5 * np.asarray(d)
    rho = np.asarray(rho)
    n0, n1 = rho.sum(), (rho * R).sum()
    n2, n3 = (rho * 4 * math.pi * R ** 2).sum(), (rho * 4 / 3 * math.pi * R ** 3).sum()
    z = np.zeros((3, 1))
    dd = dphi_hs(np.array([n0]), np.array([n1]), np.array([n2]), np.array([n3]), z, z)
    return np.array([float(dd["d0"][0] + Ri * dd["d1"][0] + 4 * math.pi * Ri ** 2 * dd["d2"][0]
                           + 4 / 3 * math.pi * Ri ** 3 * dd["d3"][0]) for Ri in R])


def spt_mu(rho, d):
    """Scaled-particle / Percus-Yevick compressibility excess chemical
    potentials of a hard-sphere mixture (Lebowitz 1964; Reiss-Frisch-Lebowitz)."""
    rho, d = np.asarray(rho, float), np.asarray(d, float)
    xi = [math.pi / 6 * float((rho * d ** m).sum()) for m in range(4)]
    one = 1.0 - xi[3]
    # beta P = (6/pi) [xi0/(1-xi3) + 3 xi1 xi2/(1-xi3)^2 + 3 xi2^3/(1-xi3)^3]
    p = 6 / math.pi * (xi[0] / one + 3 * xi[1] * xi[2] / one ** 2 + 3 * xi[2] ** 3 / one ** 3)
    return np.array([-math.log(one) + 3 * xi[2] * s / one + 3 * xi[1] * s * s / one
                     + 4.5 * xi[2] ** 2 * s * s / one ** 2 + math.pi / 6 * s ** 3 * p for s in d])


def py_single(eta):
    return -math.log(1 - eta) + (14 * eta - 13 * eta ** 2 + 5 * eta ** 3) / (2 * (1 - eta) ** 3)


@pytest.mark.parametrize("eta", [1e-4, 0.0170272018534497, 0.2, 0.45, 0.6])
def test_single_species_bulk_is_percus_yevick(eta):
    d = 0.3
    rho = eta / (math.pi / 6 * d ** 3)
    assert _bulk_mu([rho], [d])[0] == pytest.approx(py_single(eta), rel=1e-13)


def test_py_value_at_045():
    assert py_single(0.45) == pytest.approx(12.988896354624895, rel=1e-15)


def test_mixture_bulk_is_scaled_particle_theory():
    rng = np.random.default_rng(3)
    for _ in range(5):
        d = rng.uniform(0.1, 0.5, size=4)
        rho = rng.uniform(0.1, 3.0, size=4)
        assert np.allclose(_bulk_mu(rho, d), spt_mu(rho, d), rtol=1e-12, atol=0)


def test_packing_violation_raises():
    z = np.zeros((3, 1))
    with pytest.raises(ValueError):
        dphi_hs(np.ones(1), np.ones(1), np.ones(1), np.array([1.0]), z, z)


# --------------------------------------------------------------------------
# the modified (White Bear) functional
# --------------------------------------------------------------------------
from oracle import dphi_hs_wb, phi_hs_wb  # noqa: E402
from oracle.fmt import WB_SERIES_BELOW, _wb_g  # noqa: E402


@pytest.mark.parametrize("n3", [1e-4, 0.01, 0.049, 0.051, 0.2, 0.45, 0.7])
def test_wb_derivatives_match_finite_differences(n3):
    rng = np.random.default_rng(int(n3 * 1e4))
    p = _point(rng)
    p["n3"] = n3
    args = lambda q: (np.array(q["n0"]), np.array(q["n1"]), np.array(q["n2"]), np.array(q["n3"]),
                      np.asarray(q["n1v"])[:, None], np.asarray(q["n2v"])[:, None])
    d = dphi_hs_wb(*args(p))
    for key, dk in (("n0", "d0"), ("n1", "d1"), ("n2", "d2"), ("n3", "d3")):
        eps = 1e-6 * max(1e-3, abs(p[key]))
        qp, qm = dict(p), dict(p)
        qp[key] = p[key] + eps
        qm[key] = p[key] - eps
        fd = (phi_hs_wb(*args(qp)) - phi_hs_wb(*args(qm))) / (2 * eps)
        assert float(d[dk]) == pytest.approx(float(fd), rel=1e-6, abs=1e-7), key
    for key, dk in (("n1v", "d1v"), ("n2v", "d2v")):
        for c in range(3):
            eps = 1e-6
            qp, qm = dict(p), dict(p)
            qp[key] = np.array(p[key]); qp[key][c] += eps
            qm[key] = np.array(p[key]); qm[key][c] -= eps
            fd = (phi_hs_wb(*args(qp)) - phi_hs_wb(*args(qm))) / (2 * eps)
            assert float(d[dk][c]) == pytest.approx(float(fd), rel=1e-7, abs=1e-8), (key, c)


def test_wb_bracket_limits_and_switch():
    # the n2^3 coefficient tends to Rosenfeld's 1/(24 pi) at vanishing packing
    g, _ = _wb_g(np.array([0.0, 1e-8]))
    assert g[0] / 36.0 == pytest.approx(1.0 / 24.0, rel=1e-15)
    assert g[1] / 36.0 == pytest.approx(1.0 / 24.0, rel=1e-7)
    # the series and the closed form agree where they meet
    x = WB_SERIES_BELOW
    one = 1 - x
    closed = (x + one ** 2 * math.log1p(-x)) / (x ** 2 * one ** 2)
    series = sum((k + 1) * (k + 3) / (k + 2) * x ** k for k in range(40))
    assert closed == pytest.approx(series, rel=1e-12)
    gs, _ = _wb_g(np.array([x * (1 - 1e-12), x * (1 + 1e-12)]))
    assert gs[0] == pytest.approx(gs[1], rel=1e-11)


@pytest.mark.parametrize("eta", [0.1, 0.3, 0.45])
def test_wb_bulk_is_carnahan_starling(eta):
    """For a uniform one-component fluid the White Bear functional gives the
    Carnahan-Starling excess chemical potential (8 eta - 9 eta^2 + 3 eta^3) / (1 - eta)^3
    through the full evaluation (weights, derivatives, back-convolution)."""
    import oracle
    import pnp_inputs as P
    d = 0.3
    sp = [P.Species(d, 0.0, eta / (math.pi / 6.0 * d ** 3))]
    prob = P.Problem(n=8, h=0.05, species=sp, T=300.0, terms=P.TERM_HS_WB)
    rho = np.full((1, 8, 8, 8), sp[0].rho_bulk)
    mu = oracle.mu_ex(prob, rho, "fft")["total"]
    cs = (8 * eta - 9 * eta ** 2 + 3 * eta ** 3) / (1 - eta) ** 3
    assert np.max(np.abs(mu - cs)) < 1e-12 * cs
    # the Rosenfeld functional differs (it gives the Percus-Yevick value)
    ros = oracle.mu_ex(prob.with_(terms=P.TERM_HS), rho, "fft")["total"]
    assert np.max(np.abs(ros - cs)) > 1e-3 * cs


def bmcsl_mu(d, rho):
    """Excess chemical potentials of a hard-sphere mixture from the
    Boublik-Mansoori-Carnahan-Starling-Leland equation of state, written with
    xi_k = (pi/6) sum_j rho_j d_j^k (a closed form from the liquid-state
    literature, independent of any functional)."""
    d = np.asarray(d, dtype=np.float64)
    rho = np.asarray(rho, dtype=np.float64)
    x0, x1, x2, x3 = (math.pi / 6.0 * float(np.sum(rho * d ** k)) for k in range(4))
    u = 1.0 - x3
    ln = math.log(u)
    beta_p = 6.0 / math.pi * (x0 / u + 3.0 * x1 * x2 / u ** 2 + (3.0 - x3) * x2 ** 3 / u ** 3)
    out = []
    for di in d:
        a = di * x2 / x3
        out.append(-ln + (3.0 * x2 * di + 3.0 * x1 * di ** 2) / u + 4.5 * (x2 * di / u) ** 2
                   + 3.0 * a ** 2 * (ln + x3 / u - 0.5 * (x3 / u) ** 2)
                   - a ** 3 * (2.0 * ln + x3 * (2.0 - x3) / u)
                   + beta_p * math.pi * di ** 3 / 6.0)
    return np.array(out)


@pytest.mark.parametrize("rb", [(3.0, 2.0, 4.0), (0.5, 0.1, 9.0), (20.0, 1.0, 1.0)])
def test_wb_bulk_mixture_is_bmcsl(rb):
    """White Bear at uniform mixture densities, through the full evaluation,
    equals the BMCSL chemical potentials of every species."""
    import oracle
    import pnp_inputs as P
    ds = (0.15, 0.3, 0.4)
    sp = [P.Species(ds[i], 0.0, rb[i]) for i in range(3)]
    prob = P.Problem(n=8, h=0.05, species=sp, T=300.0, terms=P.TERM_HS_WB)
    got = oracle.bulk_mu_ex(prob)
    ref = bmcsl_mu(ds, rb)
    assert np.max(np.abs(got - ref)) < 1e-12 * np.max(np.abs(ref))
    # one component: Carnahan-Starling
    eta = 0.35
    one = bmcsl_mu([0.3], [eta / (math.pi / 6.0 * 0.3 ** 3)])[0]
    assert one == pytest.approx((8 * eta - 9 * eta ** 2 + 3 * eta ** 3) / (1 - eta) ** 3, rel=1e-14)
