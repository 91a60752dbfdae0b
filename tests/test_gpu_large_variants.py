"""The derivative pass's White Bear and free-energy variants on a grid that
streams its fields (192^3: the c2r steps take their mirror values through
LDS there) against the oracle's numpy-FFT route, on the channel electrolyte
with noise along all three axes: beta mu_ex per term and in total, the
Slotboom factor, and F_hs, F_el, F_sh (Sec. 2.3), in FP64 (1e-10) and mixed
precision (1e-5)."""
import numpy as np
import pytest
import torch

import oracle
import pnp_inputs as P
from conftest import relerr, to_dev

pytestmark = pytest.mark.gpu

N = 192
WB_ALL = P.TERM_HS_WB | P.TERM_EC | P.TERM_SW
_REF = {}


def _case(kind):
    if kind not in _REF:
        _REF.clear()  # one reference in host memory at a time
        if kind == "wb":
            prob, rho = P.channel_problem(N, 9601, terms=WB_ALL)
            print(f"oracle mu_ex n={N} White Bear", flush=True)
            _REF[kind] = (prob, rho, oracle.mu_ex(prob, rho, "fft"))
        else:
            prob, rho = P.channel_problem(N, 9602)
            print(f"oracle free energy n={N}", flush=True)
            _REF[kind] = (prob, rho, oracle.free_energy(prob, rho, "fft"))
    return _REF[kind]


@pytest.mark.parametrize("precision,tol", [(P.FP64, 1e-10), (P.MIXED, 1e-5)])
def test_white_bear_192(ev, precision, tol):
    prob, rho, ref = _case("wb")
    prob = prob.with_(precision=precision)
    print(f"White Bear n={N} precision={precision}", flush=True)
    rd = to_dev(rho)
    mu3, _ = ev.mu_ex(prob, rd, per_term=True, slotboom=False)
    for k, name in enumerate(("hs", "el", "sh")):
        got = mu3[k].cpu().numpy()
        for i in range(prob.S):
            assert relerr(got[i], ref[name][i]) < tol, (name, i, relerr(got[i], ref[name][i]))
    del mu3
    mu, slot = ev.mu_ex(prob, rd)
    mu, slot = mu.cpu().numpy(), slot.cpu().numpy()
    for i in range(prob.S):
        assert relerr(mu[i], ref["total"][i]) < tol, ("total", i)
    stol = tol * max(1.0, float(np.max(np.abs(ref["total"]))))
    assert float(np.max(np.abs(slot / ref["slotboom"] - 1.0))) < stol
    del rd
    torch.cuda.empty_cache()


@pytest.mark.parametrize("precision,tol", [(P.FP64, 1e-10), (P.MIXED, 1e-5)])
def test_free_energy_192(ev, precision, tol):
    prob, rho, ref = _case("fe")
    prob = prob.with_(precision=precision)
    print(f"free energy n={N} precision={precision}", flush=True)
    got, _ = ev.free_energy(prob, to_dev(rho))
    for k in ("hs", "el", "sh", "total"):
        assert abs(got[k] - ref[k]) <= tol * max(1.0, abs(ref[k])), (k, got[k], ref[k])
    torch.cuda.empty_cache()
