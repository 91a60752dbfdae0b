"""Full-size parity: the 256^3 three-species channel electrolyte at packing
0.45, evaluated exactly as the benchmark times it (mixed precision, one call,
mu_ex and Slotboom outputs), checked at 512 sampled grid points per species
against values the FP64 oracle wrote (tests/golden/cfg3_256_samples.json,
made by tests/golden/make_cfg3_samples.py), and against the FP64 GPU path
everywhere.  The same checks run at 192^3 (the largest served size, a
radix-3 grid; tests/golden/cfg3_192_samples.json).  The densities vary along
all three axes (noise and alternating-sign components on the channel).

Bars: sampled values within 1e-5 of the oracle term's largest magnitude
(per species); the mixed path within 1e-5 of the FP64 path per term
(infinity-norm relative); the FP64 path within 1e-10 at the samples.
"""
import json
import os

import numpy as np
import pytest
import torch

import pnp_inputs as P

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module", params=[256, 192])
def size(request):
    return request.param


@pytest.fixture(scope="module")
def golden(size):
    with open(os.path.join(HERE, "golden", f"cfg3_{size}_samples.json")) as f:
        return json.load(f)


@pytest.fixture(scope="module")
def workload(size):
    print(f"workload n={size}", flush=True)
    prob, rho = P.config3(n=size)
    return prob, torch.from_numpy(rho).to("cuda:0").contiguous()


def _sampled(t, idx):
    return t.reshape(t.shape[0], -1)[:, idx].cpu().numpy()


def _check(golden, mu3, tol, what):
    idx = torch.tensor(golden["flat_index"], device=mu3.device)
    for k, term in enumerate(("hs", "el", "sh")):
        got = _sampled(mu3[k], idx)
        ref = np.asarray(golden[term])
        for s in range(ref.shape[0]):
            scale = golden["max_abs"][term][s]
            err = np.max(np.abs(got[s] - ref[s])) / scale
            assert err < tol, (what, term, s, err)


def test_cfg3_mixed_as_timed(ev, golden, workload):
    prob, rho = workload
    S, n = prob.S, prob.n
    out = torch.empty((S, n, n, n), dtype=torch.float64, device=rho.device)
    slot = torch.empty_like(out)
    ev.mu_ex(prob, rho, out=out, slot=slot)          # the benchmark's call
    idx = torch.tensor(golden["flat_index"], device=rho.device)
    tot_ref = sum(np.asarray(golden[t]) for t in ("hs", "el", "sh"))
    scale = [sum(golden["max_abs"][t][s] for t in ("hs", "el", "sh")) for s in range(S)]
    got = _sampled(out, idx)
    for s in range(S):
        assert np.max(np.abs(got[s] - tot_ref[s])) / scale[s] < 1e-5, s
    got_slot = _sampled(slot, idx)
    # exp(-mu) inherits the absolute error of mu as a relative error
    rel = np.abs(got_slot / np.exp(-tot_ref) - 1.0)
    assert np.max(rel) < 1e-5 * max(scale), np.max(rel)
    del out, slot


def test_cfg3_mixed_per_term(ev, golden, workload):
    prob, rho = workload
    mu3, _ = ev.mu_ex(prob, rho, per_term=True, slotboom=False)
    _check(golden, mu3, 1e-5, "mixed")
    ref3, _ = ev.mu_ex(prob, rho, per_term=True, slotboom=False, precision=P.FP64)
    _check(golden, ref3, 1e-10, "fp64")
    for k in range(3):
        e = ((mu3[k] - ref3[k]).abs().amax(dim=(1, 2, 3)) / ref3[k].abs().amax(dim=(1, 2, 3))).cpu()
        assert float(e.max()) < 1e-5, (k, e)
    del mu3, ref3
    torch.cuda.empty_cache()


def test_on_a_callers_stream_equals_default_stream(ev, workload):
    """From 192^3 on, the Nyquist-plane tiles of the y and x passes run on the
    context's side stream, forked from and joined back into the caller's
    stream: on a non-default caller stream, with the output consumed by work
    queued after the call on that stream, the result equals the
    default-stream call bit for bit (per term and in total)."""
    prob, rho = workload
    ref, ref_slot = ev.mu_ex(prob, rho)
    ref3, _ = ev.mu_ex(prob, rho, per_term=True, slotboom=False)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        from paper_1407_0674_amd import FLAG_ASYNC
        mu, slot = ev.mu_ex(prob, rho, flags=FLAG_ASYNC, workspace=ev.workspace(ev.workspace_bytes(prob), "alt"))
        mu_c = mu.clone()   # consumed on the caller's stream right after the call
        mu3, _ = ev.mu_ex(prob, rho, per_term=True, slotboom=False)
    s.synchronize()
    assert torch.equal(mu_c, ref) and torch.equal(slot, ref_slot)
    assert torch.equal(mu3, ref3)
    del mu, slot, mu_c, mu3, ref, ref_slot, ref3
    torch.cuda.empty_cache()
