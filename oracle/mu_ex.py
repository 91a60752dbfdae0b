"""beta*mu_ex and the Slotboom factor, assembled term by term (oracle side).

Test infrastructure (see the package docstring).

Steps, in the paper's order (Sec. 2.3 and Sec. 3.4):
  1. weighted densities n_alpha = sum_i rho_i (x) omega_i^alpha   (correlation)
  2. the ten FMT derivatives dPhi/dn_alpha at every grid point
  3. beta mu_hs_i = sum_alpha dPhi/dn_alpha (*) omega_i^alpha      (convolution)
  4. beta mu_el_i = beta mu_el_i[bulk] - sum_j C_ij (*) (rho_j - rho_j^bulk)
  5. beta mu_sh_i = c_sw beta sum_j u_ij (*) rho_j, c_sw = 1/2 as printed
  6. beta mu_ex = hs + el + sh, Slotboom factor exp(-beta mu_ex) (Sec. 2.1)
All outputs are dimensionless (units of k_B T).

route="direct": kernels by explicit inverse DFT and O(N^2) sums (no FFT).
route="fft":    the same operator through numpy's real FFT.
"""
import math

import numpy as np

from .discrete import build_operator, real_space_kernel
from .direct import correlate_direct, convolve_direct
from .fmt import dphi_hs, dphi_hs_wb, phi_hs, phi_hs_wb

HS_ROSENFELD, HS_WHITE_BEAR = 1, 8  # term bits of the hard-sphere functional (Sec. 2.3.1)


def _hs_functional(terms):
    """(phi, dphi) of the selected hard-sphere free-energy density, or None."""
    if terms & HS_WHITE_BEAR:
        return phi_hs_wb, dphi_hs_wb
    if terms & HS_ROSENFELD:
        return phi_hs, dphi_hs
    return None

SCALARS = ("w0", "w1", "w2", "w3")
VECTORS = ("v1", "v2")


def _species_kernels(op):
    """Real-space kernels per species: 4 scalars, then v1 and v2 (3 comps each)."""
    ks = []
    for i in range(op.S):
        w = op.w[i]
        row = [real_space_kernel(w[a].astype(complex), op.n, op.h) for a in SCALARS]
        for v in VECTORS:
            for a in range(3):
                row.append(real_space_kernel(-1j * op.khat[a] * w[v], op.n, op.h))
        ks.append(row)
    return ks


def _unpack_n(vals):
    """vals: list of 10 arrays in the order n0..n3, n1v(xyz), n2v(xyz)."""
    return {"n0": vals[0], "n1": vals[1], "n2": vals[2], "n3": vals[3],
            "n1v": np.stack(vals[4:7]), "n2v": np.stack(vals[7:10])}


def _restrict(d, domain):
    """The derivative fields with every value outside `domain` set to zero
    (nothing changes when domain is None)."""
    if domain is None:
        return d
    m = np.asarray(domain, dtype=bool)
    return {k: np.where(m, v, 0.0) for k, v in d.items()}


def _dphi_list(d):
    return [d["d0"], d["d1"], d["d2"], d["d3"], *d["d1v"], *d["d2v"]]


def weighted_densities(problem, rho, route="direct", op=None, kernels=None):
    rho = np.asarray(rho, dtype=np.float64)
    S, n = rho.shape[0], rho.shape[1]
    if route == "direct":
        op = op or build_operator(problem, half=False)
        kernels = kernels or _species_kernels(op)
        F = np.stack([rho[i] for i in range(S) for _ in range(10)])
        K = np.stack([kernels[i][a] for i in range(S) for a in range(10)])
        out = correlate_direct(F, K, op.h).reshape(S, 10, n, n, n).sum(axis=0)
        return _unpack_n(list(out))
    op = op or build_operator(problem, half=True)
    rh = [np.fft.rfftn(rho[i]) for i in range(S)]
    vals = []
    for a in SCALARS:
        acc = sum(rh[i] * op.w[i][a] for i in range(S))
        vals.append(np.fft.irfftn(acc, s=(n, n, n), axes=(0, 1, 2)))
    for v in VECTORS:
        for c in range(3):
            # conj(-i khat v) = +i khat v
            acc = sum(rh[i] * (1j * op.khat[c] * op.w[i][v]) for i in range(S))
            vals.append(np.fft.irfftn(acc, s=(n, n, n), axes=(0, 1, 2)))
    return _unpack_n(vals)


def mu_ex(problem, rho, route="direct", drho=None, domain=None):
    """Returns a dict with 'n' (weighted densities), 'dphi', and per-term
    arrays 'hs', 'el', 'sh', 'total', 'slotboom', each (S, n, n, n).
    drho: the density deviation the EC convolution integrates (default
    rho - rho_bulk everywhere).
    domain: None, or a boolean (n, n, n) array marking the points where the
    free-energy density Phi_hs is integrated (F_hs = h^3 sum over those
    points); the derivative fields dPhi/dn_alpha are then zero elsewhere
    before the back-convolution, which is the functional derivative of that
    restricted sum.  None integrates over the whole periodic grid."""
    rho = np.asarray(rho, dtype=np.float64)
    S, n = rho.shape[0], rho.shape[1]
    terms = problem.terms
    half = route != "direct"
    op = build_operator(problem, half=half)
    zero = np.zeros_like(rho)
    res = {"hs": zero.copy(), "el": zero.copy(), "sh": zero.copy(), "n": None, "dphi": None}
    if drho is None:
        drho = rho - op.rho_bulk[:, None, None, None]
    else:
        drho = np.asarray(drho, dtype=np.float64)

    hs_fn = _hs_functional(terms)
    if route == "direct":
        kernels = _species_kernels(op) if hs_fn else None
        fields, kers, slots = [], [], []
        if hs_fn:
            nal = weighted_densities(problem, rho, "direct", op, kernels)
            d = _restrict(hs_fn[1](nal["n0"], nal["n1"], nal["n2"], nal["n3"], nal["n1v"], nal["n2v"]),
                          domain)
            res["n"], res["dphi"] = nal, d
            dl = _dphi_list(d)
            for i in range(S):
                for a in range(10):
                    fields.append(dl[a]); kers.append(kernels[i][a]); slots.append(("hs", i, 1.0))
        if terms & 2:
            for i in range(S):
                for j in range(S):
                    fields.append(drho[j])
                    kers.append(real_space_kernel(op.C_hat[i][j].astype(complex), n, op.h))
                    slots.append(("el", i, -1.0))
        if terms & 4:
            for i in range(S):
                for j in range(S):
                    fields.append(rho[j])
                    kers.append(real_space_kernel(op.u_hat[i][j].astype(complex), n, op.h))
                    slots.append(("sh", i, op.c_sw * op.beta))
        if fields:
            out = convolve_direct(np.stack(fields), np.stack(kers), op.h)
            for m, (term, i, f) in enumerate(slots):
                res[term][i] += f * out[m]
    else:
        def conv(f_hat, spec):
            return np.fft.irfftn(f_hat * spec, s=(n, n, n), axes=(0, 1, 2))
        if hs_fn:
            nal = weighted_densities(problem, rho, "fft", op)
            d = _restrict(hs_fn[1](nal["n0"], nal["n1"], nal["n2"], nal["n3"], nal["n1v"], nal["n2v"]),
                          domain)
            res["n"], res["dphi"] = nal, d
            dh = [np.fft.rfftn(x) for x in _dphi_list(d)]
            for i in range(S):
                w = op.w[i]
                acc = sum(dh[a] * w[SCALARS[a]] for a in range(4))
                for b, v in enumerate(VECTORS):
                    for c in range(3):
                        acc = acc + dh[4 + 3 * b + c] * (-1j * op.khat[c] * w[v])
                res["hs"][i] = np.fft.irfftn(acc, s=(n, n, n), axes=(0, 1, 2))
        if terms & 6:
            rh = [np.fft.rfftn(rho[j]) for j in range(S)]
            drh = [np.fft.rfftn(drho[j]) for j in range(S)]
            for i in range(S):
                if terms & 2:
                    res["el"][i] = -conv(sum(drh[j] * op.C_hat[i][j] for j in range(S)), 1.0)
                if terms & 4:
                    res["sh"][i] = op.c_sw * op.beta * conv(
                        sum(rh[j] * op.u_hat[i][j] for j in range(S)), 1.0)
    if terms & 2:
        res["el"] += op.mu_el_bulk[:, None, None, None]
    res["total"] = res["hs"] + res["el"] + res["sh"]
    with np.errstate(over="ignore"):
        res["slotboom"] = np.exp(-res["total"])
    return res


def free_energy(problem, rho, route="fft"):
    """Excess free energies in units of k_B T:
      F_hs = h^3 sum_r Phi_hs(n(r))                                  (Sec. 2.3.1)
      F_el = h^3 sum_i sum_r beta mu_el_i[bulk] drho_i
             - 1/2 h^3 sum_ij sum_r drho_i (C_ij (*) drho_j)           (Sec. 2.3.4)
      F_sh = 1/2 beta h^3 sum_ij sum_r rho_i (u_ij (*) rho_j)        (Sec. 2.3.2)
    (the constant F_el[bulk] is dropped)."""
    rho = np.asarray(rho, dtype=np.float64)
    S, n = rho.shape[0], rho.shape[1]
    op = build_operator(problem, half=True)
    h3 = op.h ** 3
    out = {"hs": 0.0, "el": 0.0, "sh": 0.0}
    hs_fn = _hs_functional(problem.terms)
    if hs_fn:
        nal = weighted_densities(problem, rho, "fft", op)
        out["hs"] = h3 * float(np.sum(hs_fn[0](nal["n0"], nal["n1"], nal["n2"], nal["n3"],
                                             nal["n1v"], nal["n2v"])))
    drho = rho - op.rho_bulk[:, None, None, None]
    if problem.terms & 2:
        drh = [np.fft.rfftn(drho[j]) for j in range(S)]
        e = 0.0
        for i in range(S):
            e += h3 * op.mu_el_bulk[i] * float(np.sum(drho[i]))
            cj = np.fft.irfftn(sum(drh[j] * op.C_hat[i][j] for j in range(S)), s=(n, n, n), axes=(0, 1, 2))
            e -= 0.5 * h3 * float(np.sum(drho[i] * cj))
        out["el"] = e
    if problem.terms & 4:
        rh = [np.fft.rfftn(rho[j]) for j in range(S)]
        e = 0.0
        for i in range(S):
            uj = np.fft.irfftn(sum(rh[j] * op.u_hat[i][j] for j in range(S)), s=(n, n, n), axes=(0, 1, 2))
            e += 0.5 * op.beta * h3 * float(np.sum(rho[i] * uj))
        out["sh"] = e
    out["total"] = out["hs"] + out["el"] + out["sh"]
    return out
