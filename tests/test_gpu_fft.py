"""GPU: the library's 3D real DFT passes against numpy's rfftn (a library
FFT) on seeded random fields, every supported size, both precisions.  From
192^3 up the spectral fields pad each kx plane (more values in FP32 than in
FP64), so the largest sizes also check the padded layout of every pass and of
the export to numpy's layout."""
import numpy as np
import pytest
import torch

from conftest import relerr, to_dev

pytestmark = pytest.mark.gpu

SIZES = [8, 16, 24, 32, 48, 64, 96, 128, 192, 256]


@pytest.mark.parametrize("n", SIZES)
@pytest.mark.parametrize("prec,tol", [(0, 1e-13), (1, 2e-6)])
def test_rfft3_matches_numpy(ev, n, prec, tol):
    rng = np.random.default_rng(n)
    x = rng.normal(size=(2, n, n, n)) + 1.5
    X = ev.rfft3(to_dev(x), prec).cpu().numpy()
    ref = np.fft.rfftn(x, axes=(1, 2, 3))
    assert X.shape == ref.shape
    for c in range(2):
        assert relerr(X[c], ref[c]) < tol


@pytest.mark.parametrize("n", SIZES)
@pytest.mark.parametrize("prec,tol", [(0, 1e-13), (1, 2e-6)])
def test_irfft3_matches_numpy(ev, n, prec, tol):
    rng = np.random.default_rng(100 + n)
    x = rng.normal(size=(1, n, n, n))
    X = np.fft.rfftn(x, axes=(1, 2, 3))
    y = ev.irfft3(to_dev(X), prec).cpu().numpy() / n ** 3
    assert relerr(y, x) < tol
