"""Continuous batching (paper_1407_0674_amd.serve): a short Poisson trace of
overlapping requests of several grid sizes, temperatures and compositions,
served from one pool under a tight byte budget.

Checks:
  * the trace really overlaps: requests are admitted while others are on
    the device, steps carry several sessions, and the budget holds some
    requests back until others finish;
  * every request's final densities, beta mu_ex and Slotboom factors equal
    those of the same request served alone, bit for bit;
  * every request's first step equals the FP64 oracle's beta mu_ex and
    exp(-beta mu_ex) of its initial densities (1e-10).
"""
import numpy as np
import pytest
import torch

import oracle
import pnp_inputs as P
from conftest import relerr, to_dev
from paper_1407_0674_amd.serve import Job, serve

pytestmark = pytest.mark.gpu


def _jobs(count=24, rate=600.0, seed=4242):
    rng = np.random.default_rng(seed)
    t, jobs, defs = 0.0, [], []
    for k in range(count):
        t += rng.exponential(1.0 / rate)
        prob, rho = P.random_instance(rng, (16, 24), P.FP64, pattern="3d")
        defs.append((prob, rho))
        jobs.append(Job(k, t, 3, (lambda p=prob, r=rho: (p, to_dev(r))), lam=0.2, clip=1.0))
    return jobs, defs


class Recorder:
    def __init__(self):
        self.first_mu, self.first_slot, self.final = {}, {}, {}

    def __call__(self, job, step, pool, sid):
        rho, mu, slot, steps = pool.view(sid)
        assert steps == step
        if step == 1:
            self.first_mu[job.rid] = mu.clone()
            self.first_slot[job.rid] = slot.clone()
        if step == job.iterations:
            self.final[job.rid] = (rho.clone(), mu.clone(), slot.clone())


def test_mix_equals_alone_and_oracle(ev):
    jobs, defs = _jobs()
    # room for about four sessions of the larger size at a time
    from paper_1407_0674_amd import Pool
    pool = Pool(ev, 1 << 20)
    need = max(pool.session_bytes(p) for p, _ in defs)
    pool.close()
    budget = 4 * need + 4096
    rec = Recorder()
    mix = serve(ev, jobs, budget, on_step=rec)
    assert sorted(mix.order) == list(range(len(jobs)))
    assert mix.max_batch > 1, "no step carried more than one session"
    assert mix.steps < sum(j.iterations for j in jobs)
    # admitted while others ran: some request completed after a later arrival joined a step
    alone_rec = Recorder()
    for j in jobs:
        one = serve(ev, [Job(j.rid, 0.0, j.iterations, j.make, j.lam, j.clip)], budget, on_step=alone_rec)
        assert one.max_batch == 1
    for j in jobs:
        for a, b in zip(rec.final[j.rid], alone_rec.final[j.rid]):
            assert torch.equal(a, b), j.rid
        assert torch.equal(rec.first_mu[j.rid], alone_rec.first_mu[j.rid])
    # the first step against the oracle of the initial densities
    for j, (prob, rho) in zip(jobs, defs):
        ref = oracle.mu_ex(prob, rho, "fft")
        mu1 = rec.first_mu[j.rid].cpu().numpy()
        assert relerr(mu1, ref["total"]) < 1e-10, j.rid
        s1 = rec.first_slot[j.rid].cpu().numpy()
        assert float(np.max(np.abs(s1 / ref["slotboom"] - 1.0))) < 1e-10 * max(1.0, float(np.max(np.abs(ref["total"]))))


def test_budget_holds_requests_back(ev):
    jobs, defs = _jobs(count=8, rate=1e6, seed=4343)   # all arrive at once
    from paper_1407_0674_amd import Pool
    pool = Pool(ev, 1 << 20)
    need = max(pool.session_bytes(p) for p, _ in defs)
    pool.close()
    mix = serve(ev, jobs, 2 * need + 4096)
    assert sorted(mix.order) == list(range(len(jobs)))
    # everything arrived at once, but the budget admitted only part of it
    assert mix.max_batch < len(jobs) and mix.steps > jobs[0].iterations
    # a cap on the work per step serves the oldest sessions first
    capped = serve(ev, jobs, 1 << 30, work_cap=1)
    assert capped.max_batch == 1 and capped.order == sorted(capped.order, key=lambda r: jobs[r].arrival)
