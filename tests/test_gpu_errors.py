"""GPU: error paths raised from device status words or host validation."""
import numpy as np
import pytest
import torch

import pnp_inputs as P
from conftest import to_dev
from paper_1407_0674_amd import PnpError

pytestmark = pytest.mark.gpu


def test_packing_violation(ev):
    prob, rho = P.channel_problem(16, 7)
    f = 1.2 / P.local_packing_max(rho, prob.species)
    with pytest.raises(PnpError) as e:
        ev.mu_ex(prob, to_dev(rho * f))
    assert e.value.status == -4


def test_nonfinite_input(ev):
    prob, rho = P.channel_problem(16, 8)
    rho = rho.copy()
    rho[1, 3, 4, 5] = np.nan
    with pytest.raises(PnpError) as e:
        ev.mu_ex(prob, to_dev(rho))
    assert e.value.status == -6


def test_overflow_of_slotboom_factor(ev):
    prob, rho = P.config1()
    eps, rout = P.uniform_well(prob.species, 60.0, 0.3)   # absurd depth -> mu_sh ~ -1e3
    prob = prob.with_(sw_eps=eps, sw_rout=rout)
    with pytest.raises(PnpError) as e:
        ev.mu_ex(prob, to_dev(rho))
    assert e.value.status == -5


def test_unsupported_size(ev):
    prob, rho = P.channel_problem(16, 9)
    prob = prob.with_(n=20)
    with pytest.raises(PnpError) as e:
        ev.mu_ex(prob, to_dev(np.zeros((3, 20, 20, 20))))
    assert e.value.status == -2


def test_workspace_too_small(ev):
    prob, rho = P.channel_problem(16, 10)
    small = torch.empty(1024, dtype=torch.uint8, device="cuda:0")
    with pytest.raises(PnpError) as e:
        ev.mu_ex(prob, to_dev(rho), workspace=small)
    assert e.value.status == -3


def test_status_is_cleared_between_calls(ev):
    prob, rho = P.channel_problem(16, 11)
    f = 1.2 / P.local_packing_max(rho, prob.species)
    with pytest.raises(PnpError):
        ev.mu_ex(prob, to_dev(rho * f))
    ev.mu_ex(prob, to_dev(rho))   # must succeed
