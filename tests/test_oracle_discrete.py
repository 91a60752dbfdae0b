"""Pins for the discrete operator: exact bulk sums, plane-wave eigenfunctions
(against the continuous transforms, not the DFT machinery), kernel realness
and the Nyquist rule for vector weights."""
import math

import numpy as np
import pytest

import oracle
import pnp_inputs as P
from oracle import transforms as tr
from oracle.discrete import build_operator, real_space_kernel, wavevectors


def _prob(n, d=(0.15, 0.30, 0.40), h=0.05):
    sp = [P.Species(di, 1.0, 0.5) for di in d]
    return P.Problem(n=n, h=h, species=sp, T=300.0, terms=P.TERM_HS)


@pytest.mark.parametrize("route", ["direct", "fft"])
def test_bulk_weighted_densities_exact(route):
    prob = _prob(8)
    rho_b = np.array([0.7, 1.1, 0.4])
    rho = np.broadcast_to(rho_b[:, None, None, None], (3, 8, 8, 8)).copy()
    nal = oracle.weighted_densities(prob, rho, route)
    R = np.array([0.075, 0.15, 0.2])
    assert np.allclose(nal["n0"], rho_b.sum(), rtol=1e-13, atol=0)
    assert np.allclose(nal["n1"], (rho_b * R).sum(), rtol=1e-13, atol=0)
    assert np.allclose(nal["n2"], (rho_b * 4 * math.pi * R ** 2).sum(), rtol=1e-13, atol=0)
    assert np.allclose(nal["n3"], (rho_b * 4 / 3 * math.pi * R ** 3).sum(), rtol=1e-13, atol=0)
    assert np.max(np.abs(nal["n1v"])) < 1e-14 and np.max(np.abs(nal["n2v"])) < 1e-14


def test_kernel_volume_sum_equals_transform_at_zero():
    n, h, a = 8, 0.05, 0.15
    _, _, _, kmag, _ = wavevectors(n, h)
    K = real_space_kernel(tr.ball_ft(kmag, a).astype(complex), n, h)
    assert h ** 3 * K.sum() == pytest.approx(4 / 3 * math.pi * a ** 3, rel=1e-13)


def _grid(n, h):
    c = np.arange(n) * h
    return np.meshgrid(c, c, c, indexing="ij")


@pytest.mark.parametrize("route", ["direct", "fft"])
@pytest.mark.parametrize("mvec", [(1, 0, 0), (1, 2, 0), (0, 1, 3), (2, -1, 1)])
def test_plane_wave_eigen(route, mvec):
    n, h = 8, 0.05
    L = n * h
    prob = _prob(n, d=(0.15, 0.30))
    kvec = 2 * math.pi * np.array(mvec) / L
    k = float(np.linalg.norm(kvec))
    X, Y, Z = _grid(n, h)
    phase = kvec[0] * X + kvec[1] * Y + kvec[2] * Z
    A = [0.2, 0.35]
    rho0 = [0.6, 0.9]
    rho = np.stack([rho0[i] + A[i] * np.cos(phase) for i in range(2)])
    nal = oracle.weighted_densities(prob, rho, route)
    R = [0.075, 0.15]
    exp = {
        "n0": sum(rho0[i] + A[i] * tr.j0(k * R[i]) * np.cos(phase) for i in range(2)),
        "n1": sum(R[i] * (rho0[i] + A[i] * tr.j0(k * R[i]) * np.cos(phase)) for i in range(2)),
        "n2": sum(4 * math.pi * R[i] ** 2 * rho0[i] + A[i] * tr.shell_ft(k, R[i]) * np.cos(phase)
                  for i in range(2)),
        "n3": sum(4 / 3 * math.pi * R[i] ** 3 * rho0[i] + A[i] * tr.ball_ft(k, R[i]) * np.cos(phase)
                  for i in range(2)),
    }
    for key, val in exp.items():
        assert np.max(np.abs(nal[key] - val)) < 1e-12 * max(1.0, np.max(np.abs(val))), key
    khat = kvec / k
    v2 = sum(A[i] * tr.shell_vec_ft(k, R[i]) for i in range(2))
    v1 = sum(A[i] * tr.shell_vec_ft(k, R[i]) / (4 * math.pi * R[i]) for i in range(2))
    for c in range(3):
        # outward vector weight: n_v = -sum_i A_i V_i(k) khat sin(k.r)
        assert np.max(np.abs(nal["n2v"][c] + v2 * khat[c] * np.sin(phase))) < 1e-12
        assert np.max(np.abs(nal["n1v"][c] + v1 * khat[c] * np.sin(phase))) < 1e-12


@pytest.mark.parametrize("route", ["direct", "fft"])
def test_plane_wave_on_nyquist_plane(route):
    # k along x at the Nyquist index: the scalar weights use |k| = pi/h, the
    # x component of the vector weights is dropped (and sin(pi x/h) = 0 on the
    # grid anyway); a y component at an ordinary index survives.
    n, h = 8, 0.05
    L = n * h
    prob = _prob(n, d=(0.30,))
    X, Y, Z = _grid(n, h)
    kvec = np.array([math.pi / h, 2 * math.pi / L, 0.0])
    k = float(np.linalg.norm(kvec))
    phase = kvec[0] * X + kvec[1] * Y
    rho = (0.5 + 0.3 * np.cos(phase))[None]
    nal = oracle.weighted_densities(prob, rho, route)
    R = 0.15
    assert np.max(np.abs(nal["n3"] - (4 / 3 * math.pi * R ** 3 * 0.5 + 0.3 * tr.ball_ft(k, R) * np.cos(phase)))) < 1e-13
    # y component: -A V khat_y sin(phase); x component: -A V khat_x sin(phase) with sin(pi x/h)... phase mixes,
    # the Nyquist rule removes the x component entirely
    assert np.max(np.abs(nal["n2v"][0])) < 1e-13
    V = 0.3 * tr.shell_vec_ft(k, R)
    assert np.max(np.abs(nal["n2v"][1] + V * (kvec[1] / k) * np.sin(phase))) < 1e-12


def test_vector_kernels_are_real_and_odd():
    n, h = 8, 0.05
    _, _, _, kmag, khat = wavevectors(n, h)
    V = tr.shell_vec_ft(kmag, 0.15)
    for c in range(3):
        K = real_space_kernel(-1j * khat[c] * V, n, h)
        Kr = np.roll(K[::-1, ::-1, ::-1], 1, axis=(0, 1, 2))
        assert np.max(np.abs(K + Kr)) < 1e-9 * np.max(np.abs(K))


def test_odd_n_has_no_nyquist():
    _, _, _, _, khat = wavevectors(7, 0.05)
    assert np.all(np.abs(khat).max(axis=(1, 2, 3)) > 0.5)
