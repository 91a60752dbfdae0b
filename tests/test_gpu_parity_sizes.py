"""GPU parity at every grid size the workloads use, on densities that vary
along all three axes (the channel tube with i.i.d. noise and alternating-sign
components: every wave-vector carries data, the three Nyquist planes
included, so the y and z components of the vector weights of Sec. 2.3.1 and
their per-axis bookkeeping meet non-zero values).

Each case compares beta mu_hs, beta mu_el and beta mu_sh per species, the
total and the Slotboom factor with the oracle's numpy-FFT route element by
element: FP64 within 1e-10 and mixed within 1e-5 (infinity-norm relative per
species and term).  The sizes cover the radix-2 plans (96 is 3 * 32, 128) and
the radix-3 plans (24, 48, 96, 192), and the grids from 192^3 up that take the
non-temporal cache policy.  The oracle result of a size is computed once and
shared by both precisions.
"""
import numpy as np
import pytest
import torch

import oracle
import pnp_inputs as P
from conftest import relerr, to_dev

pytestmark = pytest.mark.gpu

_REF = {}


def _case(n):
    """(problem, rho, oracle result) of the channel electrolyte at n^3."""
    if n not in _REF:
        prob, rho = P.channel_problem(n, 9000 + n)
        print(f"oracle n={n}", flush=True)
        _REF.clear()  # keep one size's reference in host memory at a time
        _REF[n] = (prob, rho, oracle.mu_ex(prob, rho, "fft"))
    return _REF[n]


def _check(ev, n, precision, tol):
    prob, rho, ref = _case(n)
    prob = prob.with_(precision=precision)
    print(f"n={n} precision={precision}", flush=True)
    rd = to_dev(rho)
    mu3, slot3 = ev.mu_ex(prob, rd, per_term=True)
    for k, name in enumerate(("hs", "el", "sh")):
        got = mu3[k].cpu().numpy()
        for i in range(prob.S):
            e = relerr(got[i], ref[name][i])
            assert e < tol, (n, precision, name, i, e)
    del mu3
    mu, slot = ev.mu_ex(prob, rd)
    mu, slot = mu.cpu().numpy(), slot.cpu().numpy()
    for i in range(prob.S):
        assert relerr(mu[i], ref["total"][i]) < tol, (n, precision, "total", i)
    # exp(-mu) carries the absolute error of mu as a relative error
    stol = tol * max(1.0, float(np.max(np.abs(ref["total"]))))
    assert float(np.max(np.abs(slot / ref["slotboom"] - 1.0))) < stol
    assert float(np.max(np.abs(slot3.cpu().numpy() / ref["slotboom"] - 1.0))) < stol
    del rd, slot3
    torch.cuda.empty_cache()


@pytest.mark.parametrize("n,precision,tol", [(n, p, t) for n in (24, 48, 96, 128, 192)
                                               for p, t in ((P.FP64, 1e-10), (P.MIXED, 1e-5))])
def test_sizes(ev, n, precision, tol):
    _check(ev, n, precision, tol)


@pytest.mark.parametrize("n", [96, 192])
def test_mixed_term_sum_in_k_space(ev, n):
    """The mixed path sums the three terms in k-space in FP32, before the last
    inverse transform.  Against the oracle that total is no less accurate
    than the FP64 sum of the three per-term outputs (each inverse-transformed
    on its own in FP32): the FP32 rounding comes from the transforms, whose
    error scales with the transformed field, and the summed field is no
    larger than its parts."""
    prob, rho, ref = _case(n)
    prob = prob.with_(precision=P.MIXED)
    rd = to_dev(rho)
    mu3, _ = ev.mu_ex(prob, rd, per_term=True, slotboom=False)
    sum64 = (mu3[0] + mu3[1] + mu3[2]).cpu().numpy()
    del mu3
    mu, _ = ev.mu_ex(prob, rd, slotboom=False)
    mu = mu.cpu().numpy()
    for i in range(prob.S):
        e_tot = relerr(mu[i], ref["total"][i])
        e_sum = relerr(sum64[i], ref["total"][i])
        print(f"n={n} species {i}: k-space FP32 sum {e_tot:.3e}, FP64 sum of terms {e_sum:.3e}", flush=True)
        assert e_tot < 1e-5 and e_sum < 1e-5
        assert e_tot <= 2.0 * e_sum + 1e-7, (n, i, e_tot, e_sum)
    del rd
    torch.cuda.empty_cache()
