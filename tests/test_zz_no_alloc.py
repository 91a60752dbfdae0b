"""The allocation-free evaluation (pnp_cdft_mu_ex_noalloc) against
pnp_cdft_mu_ex: the same kernels on the library's static scratch array give
the same bits.  Two calls in a row, the second with a smaller problem (the
array keeps the first call's contents); per-term and aperiodic calls; a size
beyond the array is refused with PNP_E_NOMEM and leaves the outputs alone;
a later call still agrees; a capturing stream is refused."""
import ctypes

import numpy as np
import pytest
import torch

import pnp_inputs as P
from conftest import to_dev
from paper_1407_0674_amd import FLAG_APERIODIC, PnpError
from paper_1407_0674_amd.binding import _Marshal

pytestmark = pytest.mark.gpu


def _pair(ev, prob, rho, per_term=False, flags=0):
    """(mu, slot) from pnp_cdft_mu_ex and from the allocation-free call."""
    rd = to_dev(rho)
    shape = ((3,) if per_term else ()) + rho.shape
    mu_a, slot_a = ev.mu_ex(prob, rd, per_term=per_term, flags=flags)
    mu_b = torch.full(shape, float("nan"), dtype=torch.float64, device=rd.device)
    slot_b = torch.full(rho.shape, float("nan"), dtype=torch.float64, device=rd.device)
    print(f"noalloc n={prob.n} S={prob.S} precision={prob.precision} per_term={per_term} flags={flags}", flush=True)
    ev.mu_ex_noalloc(prob, rd, mu_b, slot_b, per_term=per_term, flags=flags)
    return mu_a, slot_a, mu_b, slot_b


def test_two_calls_second_smaller(ev):
    big = P.channel_problem(64, 9501, precision=P.MIXED)
    small = P.channel_problem(32, 9502, precision=P.MIXED)
    for prob, rho in (big, small):
        mu_a, slot_a, mu_b, slot_b = _pair(ev, prob, rho)
        assert torch.equal(mu_a, mu_b)
        assert torch.equal(slot_a, slot_b)


def test_fp64_per_term_and_aperiodic(ev):
    prob, rho = P.channel_problem(48, 9503)
    mu_a, slot_a, mu_b, slot_b = _pair(ev, prob, rho, per_term=True)
    assert torch.equal(mu_a, mu_b) and torch.equal(slot_a, slot_b)
    prob, rho = P.channel_problem(16, 9504)
    mu_a, slot_a, mu_b, slot_b = _pair(ev, prob, rho, flags=FLAG_APERIODIC)
    assert torch.equal(mu_a, mu_b) and torch.equal(slot_a, slot_b)
    prob, rho = P.config1()
    mu_a, slot_a, mu_b, slot_b = _pair(ev, prob, rho)
    assert torch.equal(mu_a, mu_b) and torch.equal(slot_a, slot_b)


def test_too_large_is_refused(ev):
    prob, rho = P.channel_problem(128, 9505, precision=P.MIXED)
    assert ev.workspace_bytes(prob) > 64 << 20
    rd = to_dev(rho)
    out = torch.zeros(rho.shape, dtype=torch.float64, device=rd.device)
    with pytest.raises(PnpError) as e:
        ev.mu_ex_noalloc(prob, rd, out)
    assert e.value.status == -3
    assert float(out.abs().max()) == 0.0
    # the next call that fits still agrees with the workspace call
    prob, rho = P.channel_problem(24, 9506, precision=P.MIXED)
    mu_a, slot_a, mu_b, slot_b = _pair(ev, prob, rho)
    assert torch.equal(mu_a, mu_b) and torch.equal(slot_a, slot_b)


def test_capturing_stream_is_refused(ev):
    prob, rho = P.channel_problem(16, 9507)
    rd = to_dev(rho)
    out = torch.zeros(rho.shape, dtype=torch.float64, device=rd.device)
    m = _Marshal(prob)
    s = torch.cuda.Stream()
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=s):
        st = ev.lib.pnp_cdft_mu_ex_noalloc(ev.ctx, ctypes.byref(m.grid), m.S, m.species,
                                           ctypes.c_void_p(rd.data_ptr()), m.T, ctypes.byref(m.params),
                                           ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(0),
                                           ctypes.c_void_p(s.cuda_stream))
    assert st == -1
    torch.cuda.synchronize()
    assert float(out.abs().max()) == 0.0
