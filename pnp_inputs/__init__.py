"""Seeded synthetic workloads for the cDFT excess-chemical-potential evaluation.

This module only *describes* problems and draws their random inputs.  It holds
none of the method's arithmetic (no weights, no convolutions, no functional):
both the CPU oracle and the GPU path receive the same description and the
same density arrays from here and compute everything else on their own.

Units: nm, eV, K, number densities in nm^-3.  Concentrations quoted in mol/L
are converted with 1 M = 0.602214076 nm^-3 (Avogadro's number times 1e-24).

The species model follows the paper's charged hard spheres (Sec. 2.3: a
diameter, a valence and a bulk density per species); the square-well
attraction follows Sec. 2.3.2 (depth eps_ab on sigma_ab <= r <= r_out).
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace
from typing import List, Optional, Sequence

import numpy as np

MOLAR_TO_NM3 = 0.602214076

TERM_HS = 1
TERM_EC = 2
TERM_SW = 4
TERM_HS_WB = 8  # hard spheres with the modified (White Bear) functional instead of Rosenfeld's
TERMS_ALL = TERM_HS | TERM_EC | TERM_SW

FP64 = 0
MIXED = 1

BASE_SEED = 14070674


@dataclass(frozen=True)
class Species:
    """One species: hard-core diameter d [nm], valence q, bulk density
    rho_bulk [nm^-3], the bulk electrostatic-correlation chemical potential
    mu_el_bulk [k_B T] that the paper leaves unspecified, and whether it is
    mobile (an ion) or stationary (fixed sites, whose density the density
    updates leave alone)."""
    d: float
    q: float
    rho_bulk: float
    mu_el_bulk: float = 0.0
    mobile: bool = True


@dataclass
class Problem:
    """A complete description of one mu_ex evaluation on a periodic grid.

    sw_eps  : S x S well depths [eV] (positive = attractive), or None (no well)
    sw_rout : S x S outer well radii [nm]; entries <= 0 mean gamma * sigma_ab
    """
    n: int
    h: float
    species: List[Species]
    T: float
    terms: int = TERMS_ALL
    eps_r: float = 16.6
    sw_eps: Optional[np.ndarray] = None
    sw_rout: Optional[np.ndarray] = None
    sw_gamma: float = 1.2
    sw_prefactor: float = 0.5
    precision: int = FP64
    name: str = ""

    @property
    def S(self) -> int:
        return len(self.species)

    @property
    def shape(self):
        return (self.S, self.n, self.n, self.n)

    def with_(self, **kw) -> "Problem":
        return replace(self, **kw)


# --------------------------------------------------------------------------
# well descriptions (pure bookkeeping on the workload's own numbers)
# --------------------------------------------------------------------------

def uniform_well(species: Sequence[Species], depth_eV: float, width_nm: float):
    """Square wells of one depth for every pair, reaching `width_nm` beyond
    contact (r_out = (d_a + d_b)/2 + width)."""
    S = len(species)
    eps = np.full((S, S), float(depth_eV))
    rout = np.empty((S, S))
    for a in range(S):
        for b in range(S):
            rout[a, b] = 0.5 * (species[a].d + species[b].d) + width_nm
    return eps, rout


# --------------------------------------------------------------------------
# density patterns
# --------------------------------------------------------------------------

def uniform_noise(rng, n: int, rho_b: Sequence[float], amp: float) -> np.ndarray:
    """rho_i(r) = rho_b,i (1 + amp * U(-1, 1)), i.i.d. per point and species."""
    S = len(rho_b)
    out = np.empty((S, n, n, n))
    for i in range(S):
        out[i] = rho_b[i] * (1.0 + amp * rng.uniform(-1.0, 1.0, size=(n, n, n)))
    return out


def gaussian_channel(rng, n: int, h: float, rho_b: Sequence[float],
                     q: Sequence[float], amp: float = 0.5) -> np.ndarray:
    """A periodic Gaussian tube along y: g = exp(-d_perp^2 / (2 w^2)) with the
    minimum-image distance to a random axis (cx, cz), width w ~ U(L/10, L/6).
    Cations gather in the tube, anions are pushed out:
        rho_i = rho_b,i [1 + amp * sign(q_i) * (2 g - 1)]."""
    prof = gaussian_channel_profile(rng, n, h, rho_b, q, amp)
    return np.ascontiguousarray(np.broadcast_to(prof[:, :, None, :], (len(rho_b), n, n, n)))


def gaussian_channel_profile(rng, n: int, h: float, rho_b: Sequence[float],
                             q: Sequence[float], amp: float = 0.5) -> np.ndarray:
    """The (x, z) profile [S][n][n] of gaussian_channel (the pattern is constant
    along y); broadcasting it along y gives gaussian_channel's array exactly."""
    L = n * h
    cx, cz = rng.uniform(0.0, L, size=2)
    w = rng.uniform(L / 10.0, L / 6.0)
    c = np.arange(n) * h
    dx = c - cx
    dx -= L * np.round(dx / L)
    dz = c - cz
    dz -= L * np.round(dz / L)
    d2 = dx[:, None] ** 2 + dz[None, :] ** 2            # (x, z)
    g = np.exp(-d2 / (2.0 * w * w))
    S = len(rho_b)
    out = np.empty((S, n, n))
    for i in range(S):
        s = np.sign(q[i]) if q[i] != 0 else 0.0
        out[i] = rho_b[i] * (1.0 + amp * s * (2.0 * g - 1.0))  # (x, z)
    return out


def channel_3d(rng, n: int, h: float, rho_b: Sequence[float], q: Sequence[float],
               amp: float = 0.5, noise: float = 0.1, nyquist: float = 0.05) -> np.ndarray:
    """The Gaussian tube of gaussian_channel made to vary along all three
    axes: the tube densities times
        1 + noise * U(-1, 1) + nyquist * ((-1)^x + (-1)^y + (-1)^z) / 3,
    with the uniform draws i.i.d. per point and species.  The noise puts
    weight on every wave-vector (k_y = 0 is no longer singled out), and the
    alternating-sign terms put a sizeable share of it on the three Nyquist
    planes.  Densities stay positive for amp + noise + nyquist < 1."""
    prof = gaussian_channel_profile(rng, n, h, rho_b, q, amp)
    S = len(rho_b)
    alt = np.where(np.arange(n) % 2 == 0, 1.0, -1.0)
    stag = (alt[:, None, None] + alt[None, :, None] + alt[None, None, :]) / 3.0
    out = np.empty((S, n, n, n))
    for i in range(S):
        out[i] = prof[i][:, None, :] * (1.0 + noise * rng.uniform(-1.0, 1.0, size=(n, n, n)) + nyquist * stag)
    return out


def local_packing_max(rho: np.ndarray, species: Sequence[Species]) -> float:
    """max_r sum_i rho_i(r) * pi d_i^3 / 6: the workload's own (unsmoothed)
    packing fraction, used only to size the inputs."""
    eta = np.zeros(rho.shape[1:])
    for i, sp in enumerate(species):
        eta += rho[i] * (np.pi / 6.0) * sp.d ** 3
    return float(eta.max())


# --------------------------------------------------------------------------
# the five workloads
# --------------------------------------------------------------------------

def config1(seed: int = BASE_SEED + 1):
    """16^3, h = 0.05 nm, two hard spheres d = 0.30 nm, z = +1/-1 at 1.0 M with
    10 % i.i.d. noise, T = 300 K, HS + square well (0.3 eV, 0.3 nm), FP64."""
    rng = np.random.default_rng(seed)
    sp = [Species(0.30, +1.0, 1.0 * MOLAR_TO_NM3), Species(0.30, -1.0, 1.0 * MOLAR_TO_NM3)]
    eps, rout = uniform_well(sp, 0.3, 0.3)
    prob = Problem(n=16, h=0.05, species=sp, T=300.0, terms=TERM_HS | TERM_SW,
                   sw_eps=eps, sw_rout=rout, precision=FP64, name="cfg1-16^3-S2-fp64")
    rho = uniform_noise(rng, prob.n, [s.rho_bulk for s in sp], 0.1)
    return prob, rho


def channel_problem(n: int, seed: int, precision: int = FP64, h: float = 0.05,
                    T: float = 300.0, terms: int = TERMS_ALL, pattern: str = "3d"):
    """The three-species channel electrolyte of the 64^3 workload at any n:
    d = 0.15/0.30/0.40 nm, z = +1/-1/-3, bulk ~ U(0.5, 2.0) M, Gaussian tube
    modulation of amplitude 50 %, HS + EC + SW.
    pattern "3d" (default): the tube with 10 % i.i.d. noise and 5 %
    alternating-sign (Nyquist) components, varying along every axis
    (channel_3d); "tube": the plain tube, constant along y."""
    rng = np.random.default_rng(seed)
    d = (0.15, 0.30, 0.40)
    q = (+1.0, -1.0, -3.0)
    rb = rng.uniform(0.5, 2.0, size=3) * MOLAR_TO_NM3
    sp = [Species(d[i], q[i], float(rb[i])) for i in range(3)]
    eps, rout = uniform_well(sp, 0.3, 0.3)
    prob = Problem(n=n, h=h, species=sp, T=T, terms=terms, sw_eps=eps, sw_rout=rout,
                   precision=precision, name=f"channel-{n}^3-S3")
    if pattern == "tube":
        rho = gaussian_channel(rng, n, h, [s.rho_bulk for s in sp], q, 0.5)
    elif pattern == "3d":
        rho = channel_3d(rng, n, h, [s.rho_bulk for s in sp], q, 0.5)
    else:
        raise ValueError(f"unknown pattern {pattern!r}")
    return prob, rho


def config2(seed: int = BASE_SEED + 2, n: int = 64):
    prob, rho = channel_problem(n, seed, FP64)
    prob.name = f"cfg2-{n}^3-S3-fp64"
    return prob, rho


def config3(seed: int = BASE_SEED + 3, n: int = 256, eta_max: float = 0.45,
            precision: int = MIXED, pattern: str = "3d"):
    """Channel electrolyte at 256^3 scaled (densities and bulk alike) so that
    the largest local packing fraction is eta_max = 0.45."""
    prob, rho = channel_problem(n, seed, precision, pattern=pattern)
    f = eta_max / local_packing_max(rho, prob.species)
    sp = [Species(s.d, s.q, s.rho_bulk * f, s.mu_el_bulk) for s in prob.species]
    prob = prob.with_(species=sp, name=f"cfg3-{n}^3-S3-eta{eta_max}")
    return prob, rho * f


def random_instance(rng, n_choices, precision: int = MIXED, h: float = 0.05,
                    with_rho: bool = True, profile: bool = False, pattern: str = "tube"):
    """One uneven instance of the batched / served mixes: n from n_choices,
    T ~ U(250, 350) K, S ~ U{2,3,4}, d ~ U(0.15, 0.45) nm, bulk ~ U(0.1, 2.0) M,
    z ~ U{+-1, +-2}, channel pattern, HS + EC + SW (0.3 eV, 0.3 nm wells).
    With with_rho=False only the description is drawn (rho is None); with
    profile=True the second value is the (x, z) profile [S][n][n] instead of
    the full array (the same draws: broadcasting it along y gives rho).
    pattern "3d": the channel with noise and alternating-sign components
    (channel_3d) instead of the plain tube (not with profile=True)."""
    n = int(rng.choice(n_choices))
    T = float(rng.uniform(250.0, 350.0))
    S = int(rng.integers(2, 5))
    d = rng.uniform(0.15, 0.45, size=S)
    rb = rng.uniform(0.1, 2.0, size=S) * MOLAR_TO_NM3
    q = rng.choice(np.array([-2.0, -1.0, 1.0, 2.0]), size=S)
    sp = [Species(float(d[i]), float(q[i]), float(rb[i])) for i in range(S)]
    eps, rout = uniform_well(sp, 0.3, 0.3)
    prob = Problem(n=n, h=h, species=sp, T=T, terms=TERMS_ALL, sw_eps=eps,
                   sw_rout=rout, precision=precision, name=f"inst-{n}^3-S{S}")
    if not with_rho:
        return prob, None
    if profile:
        return prob, gaussian_channel_profile(rng, n, h, [s.rho_bulk for s in sp], list(q), 0.5)
    if pattern == "3d":
        return prob, channel_3d(rng, n, h, [s.rho_bulk for s in sp], list(q), 0.5)
    return prob, gaussian_channel(rng, n, h, [s.rho_bulk for s in sp], list(q), 0.5)


def many_species(n: int, S: int, seed: int, precision: int = FP64, h: float = 0.05, terms: int = TERMS_ALL):
    """S species (1..8) of the random-instance recipe with bulk ~ U(0.1, 1.0) M
    (lower, so that eight species stay well below close packing), 300 K,
    the three-dimensional channel pattern (channel_3d)."""
    rng = np.random.default_rng(seed)
    d = rng.uniform(0.15, 0.45, size=S)
    rb = rng.uniform(0.1, 1.0, size=S) * MOLAR_TO_NM3
    q = rng.choice(np.array([-2.0, -1.0, 1.0, 2.0]), size=S)
    sp = [Species(float(d[i]), float(q[i]), float(rb[i])) for i in range(S)]
    eps, rout = uniform_well(sp, 0.3, 0.3)
    prob = Problem(n=n, h=h, species=sp, T=300.0, terms=terms, sw_eps=eps, sw_rout=rout,
                   precision=precision, name=f"many-{n}^3-S{S}")
    return prob, channel_3d(rng, n, h, [s.rho_bulk for s in sp], list(q), 0.5)


def config4(seed: int = BASE_SEED + 4, count: int = 64, n_choices=(32, 48, 64, 96, 128),
            precision: int = MIXED):
    """64 uneven instances for one batched launch."""
    rng = np.random.default_rng(seed)
    return [random_instance(rng, n_choices, precision) for _ in range(count)]


@dataclass
class Request:
    """One served request.  Its densities are drawn lazily from its own seed
    (a 200 req/s trace would not fit in host memory if drawn up front)."""
    rid: int
    arrival: float            # seconds since the start of the trace
    seed: int
    n_choices: tuple
    precision: int
    iterations: int = 5

    def problem(self) -> Problem:
        return random_instance(np.random.default_rng(self.seed), self.n_choices,
                               self.precision, with_rho=False)[0]

    def build(self):
        return random_instance(np.random.default_rng(self.seed), self.n_choices,
                               self.precision)

    def build_profile(self):
        """(problem, (x, z) profile [S][n][n]); rho is the profile broadcast along y."""
        return random_instance(np.random.default_rng(self.seed), self.n_choices,
                               self.precision, profile=True)


def config5(seed: int = BASE_SEED + 5, rate: float = 200.0, duration: float = 10.0,
            n_choices=(48, 64, 96, 128, 192), precision: int = MIXED,
            iterations: int = 5, max_requests: Optional[int] = None):
    """Poisson arrivals at `rate` req/s over `duration` s; each request asks
    for `iterations` repeated evaluations on its own resident state."""
    rng = np.random.default_rng(seed)
    t = 0.0
    reqs = []
    while True:
        t += rng.exponential(1.0 / rate)
        if t >= duration:
            break
        if max_requests is not None and len(reqs) >= max_requests:
            break
        reqs.append(Request(len(reqs), t, int(rng.integers(0, 2**62)), tuple(n_choices),
                            precision, iterations))
    return reqs


__all__ = [
    "MOLAR_TO_NM3", "TERM_HS", "TERM_EC", "TERM_SW", "TERM_HS_WB", "TERMS_ALL", "FP64", "MIXED",
    "Species", "Problem", "Request", "uniform_well", "uniform_noise",
    "gaussian_channel", "gaussian_channel_profile", "channel_3d", "local_packing_max", "config1", "config2", "config3",
    "config4", "config5", "channel_problem", "random_instance", "many_species", "BASE_SEED",
]
