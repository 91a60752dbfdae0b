"""Write sampled oracle outputs for the 256^3 channel workload at packing 0.45.

The CPU oracle (numpy FFT route, FP64) evaluates the whole problem once; the
values of beta mu_hs, beta mu_el, beta mu_sh at 512 seeded random grid points
per species are stored, so GPU tests at the full size can compare without
re-running the oracle.  Run:  python tests/golden/make_cfg3_samples.py
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
    prob, rho = P.config3()
    res = oracle.mu_ex(prob, rho, "fft")
    rng = np.random.default_rng(777)
    n = prob.n
    idx = rng.integers(0, n ** 3, size=512)
    out = {"workload": "config3 recipe, n=256, seed default, mixed-precision problem",
           "generator": "tests/golden/make_cfg3_samples.py (oracle fft route, float64)",
           "flat_index": [int(i) for i in idx]}
    for term in ("hs", "el", "sh"):
        out[term] = [[float(v) for v in res[term][s].reshape(-1)[idx]] for s in range(prob.S)]
    out["max_abs"] = {t: [float(np.max(np.abs(res[t][s]))) for s in range(prob.S)] for t in ("hs", "el", "sh")}
    with open(os.path.join(HERE, "cfg3_256_samples.json"), "w") as f:
        json.dump(out, f, indent=0)


if __name__ == "__main__":
    main()
