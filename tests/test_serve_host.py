"""The continuous-batching loop of paper_1407_0674_amd.serve as host logic,
on the CPU: a stand-in pool with a byte budget and a simulated clock in
which a step takes time in proportion to the grid points it evaluates.

Checks: requests are admitted in arrival order while they fit the budget
(the head of the queue waits for room, so admission never reorders them),
each gets exactly its number of steps, a step takes the oldest active
sessions within the per-step cap (at least one), max_active bounds the
active set, the loop sleeps until the next arrival when idle, latency runs
from arrival to the end of the last step, and a request that cannot fit an
empty pool or a non-zero step status raises."""
import types

import pytest
import torch

import paper_1407_0674_amd.binding as binding
from paper_1407_0674_amd.serve import Job, serve


class Clock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += max(0.0, dt)


class FakePool:
    """Sessions of the request's byte size in a pool of `nbytes`; a step
    advances the clock by 1 ns per grid point plus 0.1 ms."""
    last = None

    def __init__(self, ev, nbytes):
        self.nbytes, self.used, self.next = nbytes, 0, 1
        self.sessions, self.steps, self.admitted = {}, [], []
        self.max_open = 0
        self.clock, self.bad = ev.clock, ev.bad
        FakePool.last = self

    def graphs(self, k):
        pass

    def open(self, prob, rho0, lam=0.1, clip=1.0):
        if self.used + prob.nbytes > self.nbytes:
            return None
        sid = self.next
        self.next += 1
        self.used += prob.nbytes
        self.sessions[sid] = prob
        self.admitted.append(prob.rid)
        self.max_open = max(self.max_open, len(self.sessions))
        return sid

    def step(self, ids):
        self.steps.append([self.sessions[i].rid for i in ids])
        self.clock.t += sum(self.sessions[i].n ** 3 * self.sessions[i].S for i in ids) * 1e-9 + 1e-4
        return [1 if self.sessions[i].rid in self.bad else 0 for i in ids]

    def close_session(self, sid):
        self.used -= self.sessions[sid].nbytes
        del self.sessions[sid]

    def close(self):
        pass


@pytest.fixture
def env(monkeypatch):
    monkeypatch.setattr(binding, "Pool", FakePool)
    monkeypatch.setattr(torch.cuda, "current_stream", lambda *a, **k: types.SimpleNamespace(synchronize=lambda: None))
    monkeypatch.setattr(torch.cuda, "synchronize", lambda *a, **k: None)
    clock = Clock()
    ev = types.SimpleNamespace(clock=clock, bad=set())
    return ev, clock


def _job(rid, arrival, iters, n=32, S=2, nbytes=100):
    prob = types.SimpleNamespace(rid=rid, n=n, S=S, nbytes=nbytes)
    return Job(rid, arrival, iters, lambda p=prob: (p, None))


def _run(env, jobs, budget, **kw):
    ev, clock = env
    return serve(ev, jobs, budget, clock=clock, sleep=clock.sleep, **kw), FakePool.last


def test_every_request_gets_its_steps_in_arrival_order(env):
    jobs = [_job(k, 0.0001 * k, 2 + k % 3) for k in range(8)]
    out, pool = _run(env, jobs, budget=250)  # room for two sessions at a time
    assert sorted(out.order) == list(range(8))
    assert pool.admitted == list(range(8))
    assert pool.max_open == 2
    for j in jobs:
        assert sum(step.count(j.rid) for step in pool.steps) == j.iterations
    assert out.steps == len(pool.steps)
    assert out.work == sum(j.iterations * 32 ** 3 * 2 for j in jobs)
    assert all(lat > 0 for lat in out.latency_ms)


def test_head_of_queue_waits_for_room(env):
    # request 1 needs the whole pool; request 2 would fit beside request 0
    # but must not overtake request 1
    jobs = [_job(0, 0.0, 3, nbytes=100), _job(1, 0.0001, 1, nbytes=300), _job(2, 0.0002, 1, nbytes=100)]
    out, pool = _run(env, jobs, budget=300)
    assert pool.admitted == [0, 1, 2]
    assert all(not (1 in s and 0 in s) for s in pool.steps)  # 1 admitted only after 0 left
    assert out.order.index(0) < out.order.index(1)


def test_work_cap_steps_the_oldest_sessions(env):
    jobs = [_job(k, 0.0, 2) for k in range(3)]
    w = 32 ** 3 * 2
    out, pool = _run(env, jobs, budget=1000, work_cap=2 * w)
    assert pool.steps[0] == [0, 1]
    assert all(len(s) <= 2 for s in pool.steps)
    # a cap below one session still steps one session
    out, pool = _run(env, jobs, budget=1000, work_cap=1)
    assert all(len(s) == 1 for s in pool.steps)
    assert out.max_batch == 1


def test_max_active_bounds_the_active_set(env):
    jobs = [_job(k, 0.0, 2) for k in range(4)]
    out, pool = _run(env, jobs, budget=10_000, max_active=1)
    assert pool.max_open == 1
    assert pool.steps == [[0], [0], [1], [1], [2], [2], [3], [3]]
    out, pool = _run(env, jobs, budget=10_000)
    assert pool.steps[0] == [0, 1, 2, 3]
    assert out.max_batch == 4


def test_idle_loop_sleeps_until_the_next_arrival(env):
    ev, clock = env
    jobs = [_job(0, 5.0, 1), _job(1, 9.0, 1)]
    out, pool = _run(env, jobs, budget=1000)
    step_s = 32 ** 3 * 2 * 1e-9 + 1e-4
    # each request is served alone on arrival: latency = one step
    assert out.latency_ms == pytest.approx([step_s * 1e3, step_s * 1e3])
    assert clock.t == pytest.approx(9.0 + step_s)


def test_request_larger_than_the_pool_raises(env):
    with pytest.raises(RuntimeError, match="does not fit an empty pool"):
        _run(env, [_job(0, 0.0, 1, nbytes=500)], budget=100)


def test_failed_step_raises(env):
    ev, clock = env
    ev.bad.add(1)
    with pytest.raises(RuntimeError, match="request 1: status 1"):
        _run(env, [_job(0, 0.0, 2), _job(1, 0.0, 2)], budget=1000)
