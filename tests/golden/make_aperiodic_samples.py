"""Write sampled oracle outputs of the aperiodic mode for the 128^3 domain of
the benchmark's channel electrolyte (packing 0.45), evaluated on the doubled
256^3 grid.

The CPU oracle (numpy FFT route, FP64, oracle.mu_ex_aperiodic) evaluates the
whole problem once; beta mu_hs, beta mu_el, beta mu_sh at 512 seeded random
domain points per species are stored, half of them within four grid points
of a face (where zero extension matters most), so the GPU test at this size
can compare without re-running the oracle.
Run:  python tests/golden/make_aperiodic_samples.py
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import pnp_inputs as P  # noqa: E402


def main():
    prob, rho = P.config3(n=128)
    res = oracle.mu_ex_aperiodic(prob, rho, "fft")
    rng = np.random.default_rng(778)
    n = prob.n
    inner = rng.integers(0, n ** 3, size=256)
    # near a face: one coordinate within 4 points of 0 or n - 1
    xyz = rng.integers(0, n, size=(256, 3))
    axis = rng.integers(0, 3, size=256)
    near = rng.integers(0, 4, size=256)
    side = rng.integers(0, 2, size=256)
    xyz[np.arange(256), axis] = np.where(side == 0, near, n - 1 - near)
    face = (xyz[:, 0] * n + xyz[:, 1]) * n + xyz[:, 2]
    idx = np.concatenate([inner, face])
    out = {"workload": "config3 recipe at n=128 (packing 0.45, mixed-precision problem), aperiodic mode",
           "generator": "tests/golden/make_aperiodic_samples.py (oracle.mu_ex_aperiodic, fft route, float64)",
           "flat_index": [int(i) for i in idx]}
    for term in ("hs", "el", "sh"):
        out[term] = [[float(v) for v in res[term][s].reshape(-1)[idx]] for s in range(prob.S)]
    out["max_abs"] = {t: [float(np.max(np.abs(res[t][s]))) for s in range(prob.S)] for t in ("hs", "el", "sh")}
    with open(os.path.join(HERE, "aperiodic_128_samples.json"), "w") as f:
        json.dump(out, f, indent=0)


if __name__ == "__main__":
    main()
