"""Write sampled oracle outputs for the channel workload at packing 0.45, at
256^3 (the benchmark's size) and 192^3 (the largest served size, a radix-3
grid).

The densities vary along all three axes (the tube with i.i.d. noise and
alternating-sign components, which put weight on every wave-vector including
the three Nyquist planes), so the y and z components of the vector weights
meet non-zero data.  The CPU oracle (numpy FFT route, FP64) evaluates each
whole problem once; the values of beta mu_hs, beta mu_el, beta mu_sh at 512
seeded random grid points per species are stored, so GPU tests at these
sizes can compare without re-running the oracle.
Run:  python tests/golden/make_cfg3_samples.py [n ...]   (default: 256 192)
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import pnp_inputs as P  # noqa: E402


def write(n):
    prob, rho = P.config3(n=n)
    res = oracle.mu_ex(prob, rho, "fft")
    rng = np.random.default_rng(777 if n == 256 else 777 + n)
    idx = rng.integers(0, n ** 3, size=512)
    out = {"workload": f"config3 recipe (three-dimensional channel pattern), n={n}, seed default, "
                       "packing 0.45, mixed-precision problem",
           "generator": "tests/golden/make_cfg3_samples.py (oracle fft route, float64)",
           "flat_index": [int(i) for i in idx]}
    for term in ("hs", "el", "sh"):
        out[term] = [[float(v) for v in res[term][s].reshape(-1)[idx]] for s in range(prob.S)]
    out["max_abs"] = {t: [float(np.max(np.abs(res[t][s]))) for s in range(prob.S)] for t in ("hs", "el", "sh")}
    with open(os.path.join(HERE, f"cfg3_{n}_samples.json"), "w") as f:
        json.dump(out, f, indent=0)


if __name__ == "__main__":
    for n in ([int(a) for a in sys.argv[1:]] or [256, 192]):
        write(n)
