import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: oracle cases that take tens of seconds on the CPU")


def relerr(a, b):
    """Infinity-norm relative error max|a-b| / max|b| (per array)."""
    import numpy as np
    a = np.asarray(a)
    b = np.asarray(b)
    if not (np.iscomplexobj(a) or np.iscomplexobj(b)):
        a = a.astype(np.float64)
        b = b.astype(np.float64)
    den = float(np.max(np.abs(b)))
    return float(np.max(np.abs(a - b))) / (den if den > 0 else 1.0)


@pytest.fixture(scope="session")
def ev():
    """One library context on cuda:0 (GPU tests only; fails loudly without)."""
    import torch
    from paper_1407_0674_amd import Evaluator
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    e = Evaluator(0)
    yield e
    torch.cuda.synchronize()
    e.close()


def to_dev(a):
    import torch
    return torch.from_numpy(a).to("cuda:0").contiguous()
