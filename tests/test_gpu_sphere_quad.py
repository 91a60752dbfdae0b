"""GPU sphere quadrature (pnp_sphere_quadrature, Sec. 3.5) against the oracle.

The kernel merges the k-by-k product rule and the interpolation points
(trilinear corners, or the tricubic 4 x 4 x 4 points with PNP_FLAG_CUBIC)
into one integer stencil on the host and sums it from an LDS tile; the
oracle sums the rule node by node.  Parity is element by element on small grids (ragged in
every axis against the 8 x 8 x 32 output tile, smaller than the sphere, one
point, 64 fields, every order class, both boundary modes), on sampled points
at 256^3 with the benchmark's densities and radii, and at the limits of the
LDS tile.  FP64 within 1e-12 and mixed within 1e-5 of each field's largest
scalar integral.
"""

import numpy as np
import pytest

import pnp_inputs as P
from conftest import to_dev
from oracle.sphere_quad import gaussian_bump_shell, shell_integrals, shell_integrals_at
from paper_1407_0674_amd import FLAG_APERIODIC, FLAG_CUBIC, FP64, MIXED, PnpError

pytestmark = pytest.mark.gpu

FLAG_ASYNC = 1
TOL = {FP64: 1e-12, MIXED: 1e-5}


def _compare(got, f, radii, h, k, aperiodic, tol, cubic=False):
    for i, R in enumerate(radii):
        I, Iv = shell_integrals(f[i], R, h, k, aperiodic=aperiodic, cubic=cubic)
        scale = max(float(np.max(np.abs(I))), 1e-300)
        assert np.max(np.abs(got[i, 0] - I)) / scale < tol, (i, "I")
        for a in range(3):
            assert np.max(np.abs(got[i, 1 + a] - Iv[a])) / scale < tol, (i, "xyz"[a])


def _fields(shape, F, seed):
    rng = np.random.default_rng(seed)
    return 1.0 + rng.random((F,) + tuple(shape))


@pytest.mark.parametrize("precision", [FP64, MIXED])
@pytest.mark.parametrize("aperiodic", [False, True])
def test_parity_benchmark_radii_ragged_grid(ev, precision, aperiodic):
    # the benchmark's three radii at h = 0.05 nm (R / h = 1.5, 3, 4) on a grid
    # that leaves a partial tile in every axis
    shape, h, radii, k = (20, 12, 40), 0.05, [0.075, 0.15, 0.2], 8
    f = _fields(shape, 3, 11)
    got = ev.sphere_quadrature(to_dev(f), radii, h, k, precision=precision,
                               flags=FLAG_APERIODIC if aperiodic else 0).cpu().numpy()
    _compare(got, f, radii, h, k, aperiodic, TOL[precision])


@pytest.mark.parametrize("shape,radius,k,aperiodic", [
    ((33, 17, 65), 0.17, 5, False),   # several tiles plus tails, R / h = 3.4
    ((3, 5, 2), 0.15, 4, False),      # grid smaller than the sphere: periodic images wrap twice
    ((3, 5, 2), 0.15, 4, True),
    ((1, 1, 1), 0.12, 3, False),      # one point
    ((1, 1, 1), 0.12, 3, True),
    ((16, 16, 16), 0.13, 1, False),   # order 1: a single node on the equator
    ((16, 16, 16), 0.13, 2, True),
    ((16, 16, 16), 0.13, 16, False),
])
def test_parity_shapes_and_orders(ev, shape, radius, k, aperiodic):
    h = 0.05
    f = _fields(shape, 1, 12)
    got = ev.sphere_quadrature(to_dev(f), [radius], h, k, precision=FP64,
                               flags=FLAG_APERIODIC if aperiodic else 0).cpu().numpy()
    _compare(got, f, [radius], h, k, aperiodic, TOL[FP64])


def test_parity_64_fields(ev):
    rng = np.random.default_rng(13)
    shape, h, k = (8, 9, 10), 0.05, 6
    radii = list(rng.uniform(0.02, 0.19, 64))
    f = _fields(shape, 64, 14)
    got = ev.sphere_quadrature(to_dev(f), radii, h, k, precision=FP64).cpu().numpy()
    _compare(got, f, radii, h, k, False, TOL[FP64])


@pytest.mark.parametrize("precision,ratio", [(MIXED, 6.9), (FP64, 3.9), (MIXED, 10.9), (FP64, 7.9)])
def test_largest_reach(ev, precision, ratio):
    # the largest spheres each precision's 64 KB tile takes (reach 7 and 4
    # points) and its 160 KB tile (reach 11 and 8)
    shape, h, k = (12, 10, 36), 0.05, 8
    f = _fields(shape, 2, 15)
    radii = [ratio * h, 0.5 * h]
    got = ev.sphere_quadrature(to_dev(f), radii, h, k, precision=precision).cpu().numpy()
    _compare(got, f, radii, h, k, False, TOL[precision])


@pytest.mark.parametrize("precision,aperiodic", [(MIXED, False), (FP64, False), (MIXED, True)])
def test_fullsize_sampled(ev, precision, aperiodic):
    """256^3, the benchmark's densities and radii, order 8: 384 points per field
    (a third on the faces and edges of the box, where the zero extension
    matters) against the oracle evaluated point by point."""
    import torch
    prob, rho = P.config3(n=256)
    radii = [0.5 * s.d for s in prob.species]
    rd = to_dev(rho)
    out = ev.sphere_quadrature(rd, radii, prob.h, 8, precision=precision,
                               flags=FLAG_APERIODIC if aperiodic else 0)
    rng = np.random.default_rng(16)
    n = prob.n
    pts = rng.integers(0, n, size=(384, 3))
    pts[:128, 0] = rng.choice([0, n - 1], 128)
    pts[64:128, 1] = rng.choice([0, n - 1], 64)
    idx = torch.tensor((pts[:, 0] * n + pts[:, 1]) * n + pts[:, 2], device=rd.device)
    got = out.reshape(prob.S, 4, -1)[:, :, idx].cpu().numpy()
    for i, R in enumerate(radii):
        I, Iv = shell_integrals_at(rho[i], R, prob.h, 8, pts, aperiodic=aperiodic)
        scale = float(np.max(np.abs(I)))
        assert np.max(np.abs(got[i, 0] - I)) / scale < TOL[precision], i
        for a in range(3):
            assert np.max(np.abs(got[i, 1 + a] - Iv[a])) / scale < TOL[precision], (i, a)
    del out, rd
    torch.cuda.empty_cache()


@pytest.mark.parametrize("precision", [FP64, MIXED])
@pytest.mark.parametrize("aperiodic", [False, True])
def test_cubic_parity_benchmark_radii_ragged_grid(ev, precision, aperiodic):
    shape, h, radii, k = (20, 12, 40), 0.05, [0.075, 0.15, 0.2], 8
    f = _fields(shape, 3, 21)
    flags = FLAG_CUBIC | (FLAG_APERIODIC if aperiodic else 0)
    got = ev.sphere_quadrature(to_dev(f), radii, h, k, precision=precision, flags=flags).cpu().numpy()
    _compare(got, f, radii, h, k, aperiodic, TOL[precision], cubic=True)


@pytest.mark.parametrize("shape,radius,k,aperiodic", [
    ((33, 17, 65), 0.17, 5, False),
    ((3, 5, 2), 0.15, 4, False),
    ((3, 5, 2), 0.15, 4, True),
    ((1, 1, 1), 0.12, 3, True),
    ((16, 16, 16), 0.13, 1, False),
])
def test_cubic_parity_shapes(ev, shape, radius, k, aperiodic):
    h = 0.05
    f = _fields(shape, 1, 22)
    flags = FLAG_CUBIC | (FLAG_APERIODIC if aperiodic else 0)
    got = ev.sphere_quadrature(to_dev(f), [radius], h, k, precision=FP64, flags=flags).cpu().numpy()
    _compare(got, f, [radius], h, k, aperiodic, TOL[FP64], cubic=True)


@pytest.mark.parametrize("precision,ratio", [(MIXED, 5.9), (FP64, 2.9), (MIXED, 9.9), (FP64, 6.9)])
def test_cubic_largest_reach(ev, precision, ratio):
    # one point less of radius than the trilinear stencil at each tile size
    shape, h, k = (12, 10, 36), 0.05, 8
    f = _fields(shape, 2, 23)
    radii = [ratio * h, 0.5 * h]
    got = ev.sphere_quadrature(to_dev(f), radii, h, k, precision=precision, flags=FLAG_CUBIC).cpu().numpy()
    _compare(got, f, radii, h, k, False, TOL[precision], cubic=True)


def test_cubic_gaussian_bump_fourth_order(ev):
    """With the tricubic interpolant the kernel's error against the exact
    sphere integrals of the Gaussian bump falls as h^4 (about 16x when h
    halves) and lies far below the trilinear one."""
    errs, lin = [], []
    for n in (24, 48):
        L, s, R = 4.8, 0.3, 0.25
        h = L / n
        x = h * np.arange(n)
        c = np.array([L / 2, L / 2 + 0.5 * h, L / 2 - 0.3 * h])
        X, Y, Z = np.meshgrid(x, x, x, indexing="ij")
        d = np.sqrt((X - c[0]) ** 2 + (Y - c[1]) ** 2 + (Z - c[2]) ** 2)
        f = to_dev(np.exp(-d * d / (2 * s * s))[None])
        I_ex, _ = gaussian_bump_shell(d, R, s)
        got = ev.sphere_quadrature(f, [R], h, 16, precision=FP64, flags=FLAG_CUBIC).cpu().numpy()
        errs.append(np.max(np.abs(got[0, 0] - I_ex)) / np.max(I_ex))
        got1 = ev.sphere_quadrature(f, [R], h, 16, precision=FP64).cpu().numpy()
        lin.append(np.max(np.abs(got1[0, 0] - I_ex)) / np.max(I_ex))
    assert errs[0] < 0.25 * lin[0] and errs[1] < 0.1 * lin[1]
    assert 9.0 < errs[0] / errs[1] < 25.0, errs


def test_cubic_flag_is_refused_by_the_evaluation(ev):
    prob, rho = P.channel_problem(16, 2401)
    with pytest.raises(PnpError, match="flag"):
        ev.mu_ex(prob, to_dev(rho), flags=FLAG_CUBIC)


def test_async_and_repeat_bit_identical(ev):
    import torch
    shape, h, radii, k = (24, 24, 24), 0.05, [0.075, 0.2], 8
    f = to_dev(_fields(shape, 2, 17))
    a = ev.sphere_quadrature(f, radii, h, k)
    b = ev.sphere_quadrature(f, radii, h, k, flags=FLAG_ASYNC)
    torch.cuda.synchronize()
    c = ev.sphere_quadrature(f, radii, h, k, out=torch.full_like(a, float("nan")))
    assert torch.equal(a, b) and torch.equal(a, c)


def test_gaussian_bump_against_closed_form(ev):
    """The kernel's own error against the exact sphere integrals of a Gaussian
    bump: second order in h, as the oracle's."""
    errs = []
    for n in (24, 48):
        L, s, R = 4.8, 0.3, 0.25
        h = L / n
        x = h * np.arange(n)
        c = np.array([L / 2, L / 2 + 0.5 * h, L / 2 - 0.3 * h])
        X, Y, Z = np.meshgrid(x, x, x, indexing="ij")
        d = np.sqrt((X - c[0]) ** 2 + (Y - c[1]) ** 2 + (Z - c[2]) ** 2)
        f = np.exp(-d * d / (2 * s * s))[None]
        got = ev.sphere_quadrature(to_dev(f), [R], h, 16, precision=FP64).cpu().numpy()
        I_ex, _ = gaussian_bump_shell(d, R, s)
        errs.append(np.max(np.abs(got[0, 0] - I_ex)) / np.max(I_ex))
    assert errs[0] < 0.1 and errs[1] < 0.025
    assert 3.0 < errs[0] / errs[1] < 5.5


@pytest.mark.parametrize("kwargs,match", [
    (dict(order=0), "order"),
    (dict(order=65), "order"),
    (dict(radius=[0.0]), "radius"),
    (dict(radius=[-0.1]), "radius"),
    (dict(radius=[17 * 0.05]), "radius"),
    (dict(flags=8), "flag"),
    (dict(radius=[7.2 * 0.05], precision=FP64, flags=FLAG_CUBIC), "LDS"),
    (dict(radius=[10.6 * 0.05], precision=MIXED, flags=FLAG_CUBIC), "LDS"),
    (dict(precision=7), "precision"),
    (dict(radius=[8.2 * 0.05], precision=FP64), "LDS"),
    (dict(radius=[11.6 * 0.05], precision=MIXED), "LDS"),
])
def test_errors(ev, kwargs, match):
    f = to_dev(_fields((8, 8, 8), 1, 18))
    args = dict(radius=[0.1], order=8, precision=MIXED, flags=0)
    args.update(kwargs)
    with pytest.raises(PnpError, match=match):
        ev.sphere_quadrature(f, args["radius"], 0.05, args["order"], precision=args["precision"],
                             flags=args["flags"])


def test_binding_shape_errors(ev):
    import torch
    f = to_dev(_fields((8, 8, 8), 2, 19))
    with pytest.raises(PnpError):
        ev.sphere_quadrature(f, [0.1], 0.05, 8)
    with pytest.raises(PnpError):
        ev.sphere_quadrature(f[0], [0.1], 0.05, 8)
    with pytest.raises(PnpError):
        ev.sphere_quadrature(f.float(), [0.1, 0.1], 0.05, 8)
    with pytest.raises(PnpError):
        ev.sphere_quadrature(f, [0.1, 0.1], 0.05, 8, out=torch.empty(1, device=f.device, dtype=torch.float64))


def test_runs_on_the_callers_stream(ev):
    """Work is ordered on the current (non-default) stream: an input written on
    that stream just before the call is the one integrated."""
    import torch
    shape, h, radii, k = (16, 16, 32), 0.05, [0.15], 8
    f_host = _fields(shape, 1, 20)
    ref = ev.sphere_quadrature(to_dev(f_host), radii, h, k)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        f = torch.zeros((1,) + shape, dtype=torch.float64, device="cuda:0")
        f.copy_(torch.from_numpy(f_host).to("cuda:0", non_blocking=True))
        got = ev.sphere_quadrature(f, radii, h, k, flags=FLAG_ASYNC)
    s.synchronize()
    assert torch.equal(got, ref)


def test_fullsize_agrees_with_spectral_weights(ev):
    """The two GPU routes to the delta-shell weighted densities at 256^3 with
    the benchmark's smooth channel (the plain tube, without the point-to-point
    noise of the parity inputs, which no interpolating quadrature resolves):
    n2 and n2v from the sphere quadrature (order 8, FP64) against the spectral
    weights of pnp_weighted_densities.  The densities vary over about 1 nm
    against h = 0.05 nm, so the quadrature's trilinear error stays well under
    1 % of the largest value."""
    import torch
    prob, rho = P.config3(n=256, pattern="tube")
    radii = [0.5 * s.d for s in prob.species]
    rd = to_dev(rho)
    q = ev.sphere_quadrature(rd, radii, prob.h, 8, precision=FP64)
    n2_q = q[:, 0].sum(dim=0)
    n2v_q = q[:, 1:].sum(dim=0)
    del q
    w = ev.weighted_densities(prob, rd, precision=FP64)
    n2_s, n2v_s = w[2], w[7:10]
    scale = float(n2_s.abs().max())
    e2 = float((n2_q - n2_s).abs().max()) / scale
    ev2 = float((n2v_q - n2v_s).abs().max()) / float(n2v_s.abs().max())
    assert e2 < 5e-3, e2
    assert ev2 < 2e-2, ev2
    del w, n2_q, n2v_q, rd
    torch.cuda.empty_cache()


@pytest.mark.filterwarnings("ignore:The CUDA Graph is empty")
def test_capture_is_refused(ev):
    """The stencil is copied from host memory freed on return, so the call
    refuses a capturing stream instead of recording that copy."""
    import torch
    f = to_dev(_fields((8, 8, 8), 1, 21))
    out = torch.empty((1, 4, 8, 8, 8), dtype=torch.float64, device="cuda:0")
    g = torch.cuda.CUDAGraph()
    raised = None
    with torch.cuda.graph(g):
        try:
            ev.sphere_quadrature(f, [0.1], 0.05, 8, out=out, flags=FLAG_ASYNC)
        except PnpError as e:
            raised = e
    assert raised is not None and "graph" in str(raised)
    torch.cuda.synchronize()
    ref = ev.sphere_quadrature(f, [0.1], 0.05, 8)
    assert torch.isfinite(ref).all()


def test_ring_wrap_interleaved_with_evaluations(ev):
    """Stencil records share the context's argument ring with the evaluation's
    records.  Enough asynchronous calls to wrap the ring several times,
    interleaved with evaluations, each output checked against its first call."""
    import torch
    prob, rho = P.config2()
    rd = to_dev(rho)
    mu_ref, _ = ev.mu_ex(prob, rd)
    # 48 fields at order 16 with the benchmark's radii: about 150 KB of stencil
    # records per call, so 200 calls wrap the 4 MiB ring about seven times
    shape, h, k = (16, 16, 32), 0.05, 16
    f = to_dev(_fields(shape, 48, 22))
    radii = [0.075, 0.15, 0.2] * 16
    ref = ev.sphere_quadrature(f, radii, h, k)
    outs = [torch.empty_like(ref) for _ in range(4)]
    mus = [torch.empty_like(mu_ref) for _ in range(4)]
    for it in range(200):
        ev.sphere_quadrature(f, radii, h, k, flags=FLAG_ASYNC, out=outs[it % 4])
        if it % 10 == 0:
            ev.mu_ex(prob, rd, out=mus[(it // 10) % 4])
        if it % 4 == 3:
            torch.cuda.synchronize()
            for o in outs:
                assert torch.equal(o, ref), it
    torch.cuda.synchronize()
    for m in mus:
        assert torch.equal(m, mu_ref)
