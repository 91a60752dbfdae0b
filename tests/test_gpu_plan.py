"""GPU captured evaluations (pnp_plan_*) and captured session steps.

Bars: every replay of a plan equals the batch call on the same buffers bit
for bit, also with other eager work and synchronisations between replays
and with rho rewritten in place between them; a plan with relaxation equals
batch + pnp_relax_densities step for step; a request whose evaluation raises
a status reports it from the replay and keeps its densities; a request
rejected at creation keeps its code and the others still run; a pool with
captured steps gives the same sessions as a pool without.
"""
import numpy as np
import pytest
import torch

import pnp_inputs as P
from conftest import to_dev
from paper_1407_0674_amd import Pool, bulk_mu_ex

pytestmark = pytest.mark.gpu

PACKING = -4


def _instances(seed, count, n_choices=(16, 24, 32)):
    rng = np.random.default_rng(seed)
    out = []
    for k in range(count):
        prec = P.MIXED if k % 3 else P.FP64
        out.append(P.random_instance(rng, n_choices, prec))
    return out


def _outs(rhos):
    return [torch.empty_like(r) for r in rhos], [torch.empty_like(r) for r in rhos]


def test_replays_equal_batch(ev):
    inst = _instances(31, 7)
    probs = [p for p, _ in inst]
    rhos = [to_dev(r) for _, r in inst]
    ref_mu, ref_sl, st = ev.batch(probs, rhos)
    assert st == [0] * len(inst)
    mus, sls = _outs(rhos)
    plan = ev.plan(probs, rhos, outs=mus, slots=sls)
    assert plan.created_status == [0] * len(inst)
    other_p, other_r = P.channel_problem(16, 3100)
    other_d = to_dev(other_r)
    for rep in range(4):
        for t in mus + sls:
            t.fill_(np.nan)
        plan.launch()
        assert plan.status() == [0] * len(inst)
        for k in range(len(inst)):
            assert torch.equal(mus[k], ref_mu[k]), (rep, k)
            assert torch.equal(sls[k], ref_sl[k]), (rep, k)
        ev.mu_ex(other_p, other_d)  # eager work between replays
        torch.cuda.synchronize()
    plan.close()


def test_replay_sees_rewritten_rho(ev):
    inst = _instances(32, 4, (16, 32))
    probs = [p for p, _ in inst]
    rhos = [to_dev(r) for _, r in inst]
    mus, sls = _outs(rhos)
    plan = ev.plan(probs, rhos, outs=mus, slots=sls)
    rng = np.random.default_rng(3200)
    for rep in range(3):
        for rd in rhos:
            rd.mul_(torch.from_numpy(rng.uniform(0.9, 1.1, size=tuple(rd.shape))).to(rd.device))
        plan.launch()
        assert plan.status() == [0] * len(inst)
        ref_mu, ref_sl, _ = ev.batch(probs, rhos)
        for k in range(len(inst)):
            assert torch.equal(mus[k], ref_mu[k]) and torch.equal(sls[k], ref_sl[k]), (rep, k)
    plan.close()


def test_plan_with_relax_equals_eager_steps(ev):
    inst = _instances(33, 5)
    probs = [p for p, _ in inst]
    lam, clip = 0.3, 1.0
    rho_p = [to_dev(r) for _, r in inst]
    rho_e = [r.clone() for r in rho_p]
    mus, sls = _outs(rho_p)
    mb = [bulk_mu_ex(p) for p in probs]
    plan = ev.plan(probs, rho_p, outs=mus, slots=sls, relax=[(m, lam, clip) for m in mb])
    for it in range(3):
        plan.launch()
        assert plan.status() == [0] * len(inst)
        ref_mu, ref_sl, st = ev.batch(probs, rho_e)
        assert st == [0] * len(inst)
        for p, rd, mu, m in zip(probs, rho_e, ref_mu, mb):
            ev.relax(p, rd, mu, m, lam, clip)
        torch.cuda.synchronize()
        for k in range(len(inst)):
            assert torch.equal(mus[k], ref_mu[k]), (it, k)
            assert torch.equal(rho_p[k], rho_e[k]), (it, k)
    plan.close()


def test_plan_status_and_skipped_relax(ev):
    inst = _instances(34, 3, (16, 24))
    p_bad, r_bad = inst[1]
    inst[1] = (p_bad, r_bad * (1.5 / P.local_packing_max(r_bad, p_bad.species)))
    probs = [p for p, _ in inst]
    rhos = [to_dev(r) for _, r in inst]
    before = rhos[1].clone()
    plan = ev.plan(probs, rhos, relax=[(bulk_mu_ex(p) if k != 1 else [0.0] * p.S, 0.5, 1.0)
                                        for k, p in enumerate(probs)])
    plan.launch()
    st = plan.status()
    assert st[1] == PACKING and st[0] == 0 and st[2] == 0
    assert torch.equal(rhos[1], before)  # the update was skipped on the device
    plan.close()


def test_creation_rejects_one_request(ev):
    inst = _instances(35, 3, (16,))
    probs = [p for p, _ in inst]
    rhos = [to_dev(r) for _, r in inst]
    ws = [torch.empty(ev.workspace_bytes(p), dtype=torch.uint8, device=rhos[0].device) for p in probs]
    ws[2] = torch.empty(1024, dtype=torch.uint8, device=rhos[0].device)  # too small
    mus, sls = _outs(rhos)
    plan = ev.plan(probs, rhos, outs=mus, slots=sls, workspaces=ws)
    assert plan.created_status == [0, 0, -3]
    plan.launch()
    assert plan.status() == [0, 0, -3]
    ref_mu, _, _ = ev.batch(probs[:2], rhos[:2])
    assert torch.equal(mus[0], ref_mu[0]) and torch.equal(mus[1], ref_mu[1])
    plan.close()


def test_pool_captured_steps_match_eager(ev):
    inst = _instances(36, 4, (16, 24))
    pools = [Pool(ev, 1 << 30), Pool(ev, 1 << 30)]
    pools[1].graphs(2)
    ids = [[pl.open(p, to_dev(r), lam=0.25) for p, r in inst] for pl in pools]
    schedule = [[0, 1, 2, 3], [0, 1, 2, 3], [1, 3], [0, 1, 2, 3], [2], [1, 3], [2]]
    for sel in schedule:
        for pl, idl in zip(pools, ids):
            assert pl.step([idl[k] for k in sel]) == [0] * len(sel)
        for k in range(len(inst)):
            a = pools[0].view(ids[0][k])
            b = pools[1].view(ids[1][k])
            assert a[3] == b[3]
            for x, y in zip(a[:3], b[:3]):
                assert torch.equal(x, y), (sel, k)
    pools[1].close_session(ids[1][1])  # drops the graphs that hold it
    assert pools[1].step([ids[1][3]]) == [0]
    torch.cuda.synchronize()
    for pl in pools:
        pl.close()
