"""The seeded generators: the three-dimensional channel pattern that the
parity cases and the benchmark use is not constant along any axis and puts
weight on every Nyquist plane; densities stay positive; the same seed gives
the same arrays."""
import numpy as np
import pytest

import pnp_inputs as P


@pytest.mark.parametrize("n", [16, 24])
def test_channel_varies_along_every_axis(n):
    prob, rho = P.channel_problem(n, 9000 + n)
    for ax in (1, 2, 3):
        assert float(np.max(np.ptp(rho, axis=ax))) > 0.05 * float(np.max(rho))
    f = np.abs(np.fft.fftn(rho[0]))
    h = n // 2
    for plane in (f[h, :, :], f[:, h, :], f[:, :, h]):
        assert float(plane.sum()) > 0.01 * float(f.sum())
    assert float(rho.min()) > 0.0


def test_tube_pattern_is_constant_along_y():
    prob, rho = P.channel_problem(16, 5, pattern="tube")
    assert float(np.max(np.ptp(rho, axis=2))) == 0.0


def test_seeded():
    a = P.channel_problem(16, 77)[1]
    b = P.channel_problem(16, 77)[1]
    assert np.array_equal(a, b)
    c = P.config3(n=16)
    assert abs(P.local_packing_max(c[1], c[0].species) - 0.45) < 1e-12
