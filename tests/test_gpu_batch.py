"""GPU batch path: independent requests of different sizes, species counts,
temperatures and precisions evaluated in shared launches (one grid of
workgroups spans every request of one grid size and precision).

Bars: a request evaluated in a batch equals the same request evaluated alone
bit for bit (same kernels, same per-request arithmetic); against the oracle the
usual tolerances (FP64 1e-10, mixed 1e-5, infinity-norm relative per species);
a failing request reports its own status and leaves the others untouched.
"""
import numpy as np
import pytest
import torch

import oracle
import pnp_inputs as P
from conftest import relerr, to_dev

pytestmark = pytest.mark.gpu

PACKING = -4


def _mixed_instances(seed, count, n_choices):
    rng = np.random.default_rng(seed)
    out = []
    for k in range(count):
        prec = P.MIXED if k % 3 else P.FP64
        out.append(P.random_instance(rng, n_choices, prec))
    return out


def _alone(ev, prob, rho_d):
    mu, slot = ev.mu_ex(prob, rho_d)
    return mu.clone(), slot.clone()


def test_batch_equals_alone_small(ev):
    inst = _mixed_instances(11, 9, (16, 24, 32))
    rhos = [to_dev(r) for _, r in inst]
    mus, slots, st = ev.batch([p for p, _ in inst], rhos)
    assert st == [0] * len(inst)
    for (p, _), rd, mu, sl in zip(inst, rhos, mus, slots):
        m1, s1 = _alone(ev, p, rd)
        assert torch.equal(mu, m1), p.name
        assert torch.equal(sl, s1), p.name


def test_batch_large_and_small_sizes(ev):
    """A 192^3 instance (on the caller's stream, its Nyquist tiles on the
    side stream) in one batch with instances of three smaller sizes (each
    size on a branch stream of its own): every instance equals its single
    call bit for bit, and a second batch call gives the same bits."""
    rng = np.random.default_rng(17)
    inst = [P.random_instance(rng, (192,), P.MIXED)]
    inst += [P.random_instance(rng, (n,), P.MIXED if k % 2 else P.FP64) for k, n in enumerate((16, 24, 32, 16))]
    rhos = [to_dev(r) for _, r in inst]
    mus, slots, st = ev.batch([p for p, _ in inst], rhos)
    assert st == [0] * len(inst)
    mus = [m.clone() for m in mus]
    slots = [s_.clone() for s_ in slots]
    for (p, _), rd, mu, sl in zip(inst, rhos, mus, slots):
        m1, s1 = _alone(ev, p, rd)
        assert torch.equal(mu, m1), p.name
        assert torch.equal(sl, s1), p.name
    mus2, slots2, st2 = ev.batch([p for p, _ in inst], rhos)
    assert st2 == [0] * len(inst)
    for a, b in zip(mus, mus2):
        assert torch.equal(a, b)


def test_batch_vs_oracle(ev):
    inst = _mixed_instances(12, 5, (16, 24))
    mus, slots, st = ev.batch([p for p, _ in inst], [to_dev(r) for _, r in inst])
    assert st == [0] * len(inst)
    for (p, rho), mu, sl in zip(inst, mus, slots):
        ref = oracle.mu_ex(p, rho, "fft")
        tol = 1e-10 if p.precision == P.FP64 else 1e-5
        mu, sl = mu.cpu().numpy(), sl.cpu().numpy()
        for i in range(p.S):
            assert relerr(mu[i], ref["total"][i]) < tol, (p.name, i)
            assert relerr(sl[i], ref["slotboom"][i]) < tol, (p.name, i)


def test_batch_bad_request_isolated(ev):
    inst = _mixed_instances(13, 4, (16, 24))
    p_bad, r_bad = inst[1]
    # scale one request's densities until some local packing fraction exceeds 1
    f = 1.5 / P.local_packing_max(r_bad, p_bad.species)
    inst[1] = (p_bad, r_bad * f)
    rhos = [to_dev(r) for _, r in inst]
    mus, slots, st = ev.batch([p for p, _ in inst], rhos)
    assert st[1] == PACKING
    for k in (0, 2, 3):
        assert st[k] == 0
        m1, s1 = _alone(ev, inst[k][0], rhos[k])
        assert torch.equal(mus[k], m1) and torch.equal(slots[k], s1)


def test_batch_empty(ev):
    mus, slots, st = ev.batch([], [])
    assert mus == [] and st == []


def test_config4_batch(ev):
    """The 64-instance uneven mix (n from 32 to 128, S from 2 to 4, mixed
    precision): batch equals alone for every instance; against the oracle,
    the instance with the most species of every grid size."""
    inst = P.config4()
    rhos = [to_dev(r) for _, r in inst]
    mus, slots, st = ev.batch([p for p, _ in inst], rhos)
    assert st == [0] * len(inst)
    for (p, _), rd, mu, sl in zip(inst, rhos, mus, slots):
        m1, s1 = _alone(ev, p, rd)
        assert torch.equal(mu, m1), p.name
        assert torch.equal(sl, s1), p.name
    per_size = {}
    for k, (p, _) in enumerate(inst):
        if p.n not in per_size or p.S > inst[per_size[p.n]][0].S:
            per_size[p.n] = k
    assert sorted(per_size) == [32, 48, 64, 96, 128]
    for n, k in sorted(per_size.items()):
        p, rho = inst[k]
        print(f"oracle n={n} S={p.S}", flush=True)
        ref = oracle.mu_ex(p, rho, "fft")
        mu, sl = mus[k].cpu().numpy(), slots[k].cpu().numpy()
        for i in range(p.S):
            assert relerr(mu[i], ref["total"][i]) < 1e-5, (p.name, i)
        stol = 1e-5 * max(1.0, float(np.max(np.abs(ref["total"]))))
        assert float(np.max(np.abs(sl / ref["slotboom"] - 1.0))) < stol, p.name


@pytest.mark.parametrize("lam,clip", [(0.0, 0.0), (0.1, 0.0), (1.0, 0.0), (0.5, 1.0), (1.0, 0.3)])
def test_relax_vs_oracle(ev, lam, clip):
    prob, rho = P.channel_problem(24, 5100)
    rng = np.random.default_rng(5101)
    mu = rng.normal(scale=2.0, size=rho.shape)
    mu_b = rng.normal(size=prob.S)
    rd, md = to_dev(rho), to_dev(mu)
    ev.relax(prob, rd, md, mu_b, lam, clip)
    ref = oracle.relax_densities(rho, mu, [s.rho_bulk for s in prob.species], mu_b, lam, clip)
    got = rd.cpu().numpy()
    assert np.max(np.abs(got - ref) / np.abs(ref)) < 1e-14
