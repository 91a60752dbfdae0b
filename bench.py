"""Throughput of the FFT evaluation of cDFT excess chemical potentials on one GPU.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload cfg3|cfg2]

A step is one evaluation of beta mu_ex (all nine passes: weighted densities,
FMT derivatives, back-convolution, electrostatic-correlation and square-well
terms, Slotboom factors) of one synthetic problem whose densities are already
resident in HBM.  The default workload is the 256^3 three-species channel
electrolyte at packing fraction 0.45 in mixed precision (FP32 FFTs and weight
multiplies, FP64 derivatives and accumulation).  One JSON line is printed.

Besides throughput the line carries: the roofline of the dominant kernel
(algorithmic bytes over its average duration, timed with HIP events on the
evaluation's stream inside the timed region), p50/p99 latency of synchronous
single evaluations for the mixed path and the plain FP64 path on the same
GPU, the mixed path's error against the FP64 path per term, and the CPU
oracle timed on a bounded sample of the same workload.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
F = 10  # weighted-density fields


def pass_bytes_per_point(S: int, precision: int, slot: bool = True):
    """Algorithmic HBM bytes per grid point of each pass: every pass reads its
    inputs once and writes its outputs once; a half spectrum of one field
    holds n^3/2 complex values (ts bytes per grid point and field, ts = 4 in
    the mixed path, 8 in FP64); densities in and mu / exp(-mu) out are FP64."""
    c = 4 if precision == 1 else 8
    out = 16 if slot else 8
    return {
        "z_fwd_rho": (8 + c) * S,
        "y_fwd_rho": 2 * c * S,
        "x_fwd_weights": c * S + c * F,
        "y_inv_n": 2 * c * F,
        "z_deriv": 2 * c * F,
        "y_fwd_dphi": 2 * c * F,
        "x_back_pairs": c * F + 2 * c * S,
        "y_inv_mu": 2 * c * S,
        "z_inv_final": c * S + out * S,
    }


def percentile(xs, q):
    import numpy as np
    return float(np.percentile(np.asarray(xs), q))


def workload(name):
    import pnp_inputs as P
    if name == "cfg3":
        prob, rho = P.config3()
        return prob, rho, "channel electrolyte 256^3, S=3 (d=0.15/0.30/0.40 nm, z=+1/-1/-3), " \
                          "eta_max=0.45, HS+EC+SW, mixed precision"
    if name == "cfg2":
        prob, rho = P.config2()
        return prob, rho, "channel electrolyte 64^3, S=3, HS+EC+SW, FP64"
    raise SystemExit(f"unknown workload {name}")


def time_async(ev, prob, rho_d, out, slot, steps, precision):
    import torch
    from paper_1407_0674_amd import FLAG_ASYNC
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        ev.mu_ex(prob, rho_d, out=out, slot=slot, flags=FLAG_ASYNC, precision=precision)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ev.read_status()
    return (t1 - t0) * 1e3 / steps


def latencies(ev, prob, rho_d, out, slot, reps, precision):
    import torch
    lat = []
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ev.mu_ex(prob, rho_d, out=out, slot=slot, precision=precision)   # waits for its status
        lat.append((time.perf_counter() - t0) * 1e3)
    return lat


def cpu_baseline(prob, rho):
    """The oracle (numpy FFT route, as written, FP64) timed on one evaluation
    of the benchmark's own problem, limited to one thread."""
    import oracle
    from threadpoolctl import threadpool_limits
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        oracle.mu_ex(prob, rho, "fft")
        dt = time.perf_counter() - t0
    return {"value": prob.n ** 3 * prob.S / dt, "unit": "grid-pt*species/s", "cores": 1,
            "kind": "oracle",
            "sample": f"one full evaluation of the same problem ({prob.n}^3, S={prob.S}, all terms) "
                      f"with the oracle's numpy-FFT route in FP64 on one host thread, {dt:.1f} s"}


def copy_bandwidth(ev, gib=1.0, reps=10):
    """Achievable HBM bandwidth: the library's streaming copy kernel over a
    buffer of `gib` GiB, read once and written once per launch (HIP events on
    the launching stream)."""
    import torch
    words = int(gib * (1 << 30)) // 8
    a = torch.ones(words, dtype=torch.float64, device="cuda:0")
    b = torch.empty_like(a)
    ev.copy(a, b)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        ev.copy(a, b)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    ok = bool(torch.equal(a, b))
    del a, b
    return {"GBps": 2 * words * 8 / 1e9 / (ms / 1e3), "bytes_per_launch": 2 * words * 8, "ms": ms, "verified": ok}


def traffic_from_profile(kernel, launches_per_step):
    """HBM bytes per launch of `kernel` measured by the memory counters, as
    recorded with the hash of the kernel sources they were taken on; null when
    the sources have changed since."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    h = hashlib.sha256()
    for rel in rec.get("sources", []):
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    if h.hexdigest() != rec.get("sha256"):
        return None
    k = rec.get("kernels", {}).get(kernel)
    return None if k is None else k["bytes_per_launch"]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="cfg3")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--latency-reps", type=int, default=20)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run the copy kernel (reference for the memory counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build evaluates on one GPU; --gpus must be 1 "
                                   "(independent instances shard with no communication, see DESIGN.md)"}))
        sys.exit(2)

    import numpy as np
    import torch
    from paper_1407_0674_amd import Evaluator, PASS_NAMES

    dev = torch.device("cuda:0")
    ev = Evaluator(0)
    if args.calibrate_copy:
        print(json.dumps({"copy_kernel": copy_bandwidth(ev, 1.0, 5)}), flush=True)
        ev.close()
        return
    prob, rho, desc = workload(args.workload)
    rho_d = torch.from_numpy(rho).to(dev).contiguous()
    S, n = prob.S, prob.n
    n3 = n ** 3
    out = torch.empty((S, n, n, n), dtype=torch.float64, device=dev)
    slot = torch.empty_like(out)
    prec = prob.precision

    # warmup, then the timed region with pass timing on
    ev.mu_ex(prob, rho_d, out=out, slot=slot)
    for _ in range(args.warmup):
        ev.mu_ex(prob, rho_d, out=out, slot=slot)
    ev.profile(True)
    ev.profile_read(reset=True)
    ms = time_async(ev, prob, rho_d, out, slot, args.steps, prec)
    passes = ev.profile_read(reset=True)
    ev.profile(False)
    print(json.dumps({"progress": "timed region done", "ms_per_step": ms}), file=sys.stderr, flush=True)

    lat = latencies(ev, prob, rho_d, out, slot, args.latency_reps, prec)

    bpp = pass_bytes_per_point(S, prec)
    per_pass = {}
    for name, (tot, cnt) in passes.items():
        if cnt == 0:
            continue
        avg = tot / cnt
        entry = {"avg_ms": avg, "launches": cnt}
        if name in bpp:
            gb = bpp[name] * n3 / 1e9
            entry["alg_GB"] = gb
            entry["GBps"] = gb / (avg / 1e3)
        per_pass[name] = entry
    dom = max((k for k in per_pass if k in bpp), key=lambda k: per_pass[k]["avg_ms"])
    total_bytes = sum(bpp.values()) * n3
    kernel_ms = sum(v["avg_ms"] for v in per_pass.values())

    result_fp64 = {}
    errs = {}
    if not args.no_fp64 and prec == 1:
        out64 = torch.empty_like(out)
        slot64 = torch.empty_like(out)
        ev.mu_ex(prob, rho_d, out=out64, slot=slot64, precision=0)
        ms64 = time_async(ev, prob, rho_d, out64, slot64, max(3, args.steps // 3), 0)
        lat64 = latencies(ev, prob, rho_d, out64, slot64, max(5, args.latency_reps // 2), 0)
        result_fp64 = {"ms_per_step": ms64, "p50_ms": percentile(lat64, 50), "p99_ms": percentile(lat64, 99),
                       "value": n3 * S / (ms64 / 1e3)}
        del out64, slot64
        # per-term error of the mixed path against the FP64 path (infinity-norm relative)
        m3, _ = ev.mu_ex(prob, rho_d, per_term=True, slotboom=False)
        r3, _ = ev.mu_ex(prob, rho_d, per_term=True, slotboom=False, precision=0)
        for k, name in enumerate(("hs", "el", "sh")):
            e = (m3[k] - r3[k]).abs().amax(dim=(1, 2, 3)) / r3[k].abs().amax(dim=(1, 2, 3))
            errs[name] = [float(x) for x in e.cpu()]
        del m3, r3
        torch.cuda.synchronize()

    copy = copy_bandwidth(ev)
    torch.cuda.synchronize()
    cpu = None if args.no_cpu else cpu_baseline(prob, rho)

    value = n3 * S / (ms / 1e3)
    line = {
        "metric": "mu_ex grid-pts*species/s + HBM GB/s %peak; p50/p99 solve latency vs plain FP64",
        "value": value,
        "unit": "grid-pt*species/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 FFT/weights + f64 derivatives/accumulation" if prec == 1 else "f64",
        "data": "synthetic (seeded)",
        "config": {"workload": desc, "grid": n, "species": S, "global_batch": 1,
                   "precision": "mixed" if prec == 1 else "fp64"},
        "hbm": {"model_bytes_per_step": total_bytes, "GBps": total_bytes / 1e9 / (ms / 1e3),
                "pct_peak": 100.0 * total_bytes / 1e9 / (ms / 1e3) / HBM_PEAK_GBS,
                "kernel_ms_per_step": kernel_ms, "copy_kernel_GBps": copy["GBps"],
                "pct_of_copy": 100.0 * total_bytes / 1e9 / (ms / 1e3) / copy["GBps"]},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": per_pass[dom]["GBps"], "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": per_pass[dom]["GBps"] / HBM_PEAK_GBS,
                     "traffic": traffic_from_profile(dom, 1),
                     "alg_bytes_per_launch": per_pass[dom]["alg_GB"] * 1e9},
        "latency_ms": {"p50": percentile(lat, 50), "p99": percentile(lat, 99)},
        "fp64_path": result_fp64,
        "speedup_vs_fp64": (result_fp64["ms_per_step"] / ms) if result_fp64 else None,
        "err_vs_fp64_per_term": errs,
        "passes": per_pass,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)
    ev.close()


if __name__ == "__main__":
    main()
