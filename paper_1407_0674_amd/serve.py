"""Continuous batching of mu_ex requests over resident sessions (host-side
scheduling only; every device operation goes through the C ABI's pool and
session calls).

A request asks for `iterations` repeated evaluations on its own resident
state: the consumer-stub loop of a PNP solver, one beta mu_ex evaluation and
one density relaxation per step (Sec. 3.2 relaxes the iterates between
solves).  The loop

  * admits arrived requests in arrival order while their session fits the
    pool's byte budget (the head of the queue waits for room, so admission
    never reorders requests), up to `max_active` at a time;
  * steps the oldest active sessions together in one pnp_session_step (their
    evaluations share launches per grid size), taking sessions in admission
    order while their summed grid-pt*species stays within `work_cap` (at
    least one; all active sessions when it is None);
  * retires a request after its last step and releases its block, so
    requests that arrive while others are on the device join the next step.

The arithmetic of a session does not depend on which other sessions share
its steps (launches grouped by size run the same kernels per instance), so a
request's results are the same alone and in any mix.
"""
import collections
import time
from dataclasses import dataclass, field
from typing import Callable, List, Optional, Sequence


@dataclass
class Job:
    """One request: arrival time [s] from the start of the trace, the number
    of steps, and make() -> (problem, rho0), rho0 a float64 CUDA tensor
    [S][n][n][n] that the session copies at admission."""
    rid: int
    arrival: float
    iterations: int
    make: Callable
    lam: float = 0.1
    clip: float = 1.0


@dataclass
class Served:
    latency_ms: List[float] = field(default_factory=list)   # arrival to completion, per request (completion order)
    order: List[int] = field(default_factory=list)          # request ids in completion order
    makespan_s: float = 0.0
    work: int = 0                                           # evaluated grid-pt*species
    steps: int = 0                                          # pnp_session_step calls
    max_batch: int = 0                                      # most sessions in one step


def serve(ev, jobs: Sequence[Job], budget: int, max_active: Optional[int] = None,
          work_cap: Optional[int] = None, graphs: int = 0, on_step=None, clock=time.perf_counter,
          sleep=time.sleep, progress=None) -> Served:
    """Replay `jobs` (sorted by arrival) against a pool of `budget` bytes.
    on_step(job, step, pool, sid), if given, runs after each completed step of
    a session (step counts from 1; the session is still open, also after its
    last step).  graphs > 0 replays steps from captured graphs (the pool
    keeps that many id lists).  progress(dict), if given, is called about
    every five seconds."""
    import torch
    from .binding import Pool
    pool = Pool(ev, budget)
    try:
        if graphs:
            pool.graphs(graphs)
        pending = collections.deque(sorted(jobs, key=lambda j: j.arrival))
        active = collections.OrderedDict()  # sid -> [job, steps left, problem, steps done]
        out = Served()
        t0 = clock()
        last_note = t0
        limit = max_active if max_active is not None else 1 << 30
        while pending or active:
            now = clock() - t0
            while pending and pending[0].arrival <= now and len(active) < limit:
                job = pending[0]
                prob, rho0 = job.make()
                sid = pool.open(prob, rho0, lam=job.lam, clip=job.clip)
                if sid is None:
                    if not active:
                        raise RuntimeError(f"request {job.rid} does not fit an empty pool of {budget} bytes")
                    break  # the head of the queue waits for room
                pending.popleft()
                active[sid] = [job, job.iterations, prob, 0]
            if not active:
                sleep(max(0.0, pending[0].arrival - (clock() - t0)))
                continue
            ids, acc = [], 0
            for sid, (job, left, prob, done) in active.items():  # admission order
                w = prob.n ** 3 * prob.S
                if ids and work_cap is not None and acc + w > work_cap:
                    break
                ids.append(sid)
                acc += w
            st = pool.step(ids)
            torch.cuda.current_stream().synchronize()
            out.steps += 1
            out.max_batch = max(out.max_batch, len(ids))
            done_t = clock() - t0
            for sid, s_ in zip(ids, st):
                job, left, prob, done = active[sid]
                if s_ != 0:
                    raise RuntimeError(f"request {job.rid}: status {s_}")
                out.work += prob.n ** 3 * prob.S
                left -= 1
                done += 1
                if on_step is not None:
                    on_step(job, done, pool, sid)
                if left == 0:
                    out.latency_ms.append((done_t - job.arrival) * 1e3)
                    out.order.append(job.rid)
                    pool.close_session(sid)
                    del active[sid]
                else:
                    active[sid][1] = left
                    active[sid][3] = done
            if progress is not None and clock() - last_note > 5.0:
                last_note = clock()
                progress({"done": len(out.latency_ms), "active": len(active), "pending": len(pending)})
        out.makespan_s = clock() - t0
        torch.cuda.synchronize()
        return out
    finally:
        pool.close()
