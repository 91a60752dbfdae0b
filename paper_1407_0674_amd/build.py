"""Build the HIP library libpnpcdft.so in-tree for gfx950.

    python -m paper_1407_0674_amd.build

Sources (csrc/):
  * pnp_api.hip   the C ABI (host driver) with the kernels outside the FFT
                  passes and the sphere quadrature;
  * pnp_ops.hip   the pass kernels and their launch tables, compiled once
                  per (precision, grid size, FFT schedule) with -DPNP_OPS_T /
                  -DPNP_OPS_N / -DPNP_OPS_SCHED, so they compile in parallel;
  * pnp_serve.cpp the host-only serving layer over the ABI.
Objects go to paper_1407_0674_amd/_build/ and are linked into the library.
Packed-FP32 instructions are disabled for every device pass.
"""
import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libpnpcdft.so")
OBJ = os.path.join(HERE, "_build")
SIZES = (8, 16, 24, 32, 48, 64, 96, 128, 192, 256)
PRECISIONS = ("float", "double")

HIP_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def _units():
    """(object path, extra compiler arguments, source) of every translation unit."""
    units = [(os.path.join(OBJ, "pnp_api.o"), [], os.path.join(CSRC, "pnp_api.hip")),
             (os.path.join(OBJ, "pnp_serve.o"), [], os.path.join(CSRC, "pnp_serve.cpp"))]
    for t in PRECISIONS:
        for n in SIZES:
            for sched in (0, 1):
                units.append((os.path.join(OBJ, f"pnp_ops_{t}_{n}_s{sched}.o"),
                              [f"-DPNP_OPS_T={t}", f"-DPNP_OPS_N={n}", f"-DPNP_OPS_SCHED={sched}"],
                              os.path.join(CSRC, "pnp_ops.hip")))
    return units


def _compile(unit, verbose):
    obj, extra, src = unit
    cmd = [hipcc(), *HIP_FLAGS, *extra, "-I", os.path.join(ROOT, "include"), "-c", src, "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    return cmd, res


def build(verbose: bool = False, jobs: int = 0) -> str:
    os.makedirs(OBJ, exist_ok=True)
    units = _units()
    jobs = jobs or max(1, min(16, os.cpu_count() or 1))
    with ThreadPoolExecutor(max_workers=jobs) as pool:
        results = list(pool.map(lambda u: _compile(u, verbose), units))
    failed = [(cmd, res) for cmd, res in results if res.returncode != 0]
    for cmd, res in failed:
        sys.stderr.write(" ".join(cmd) + "\n" + res.stdout + res.stderr)
    if failed:
        raise RuntimeError(f"hipcc failed on {len(failed)} translation unit(s)")
    tmp = LIB + ".tmp"
    cmd = [hipcc(), *HIP_FLAGS, "-shared", *[u[0] for u in units], "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("link failed")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
