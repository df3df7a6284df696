"""Benchmark: path-steps/s with Greeks of the Heston/Milstein Monte-Carlo path on one MI355X.

One step = one pass of the whole path over one batch: the arithmetic-average
Asian call (daily fixings), 2^20 paths x 252 Milstein steps, FP32 path state
with FP64 cross-path sums, Philox normals, price + pathwise Delta/Rho + five
central bump Greeks (Delta, Gamma, Vega, Rho, Theta) on common random numbers,
all estimators reduced across paths and copied to the host.  Inputs are
parameters only (nothing to stage); the timed region covers the library call.

Prints ONE JSON line (rank 0).  Also reported: the roofline of the path kernel
(operation-count model), the Sobol + Brownian-bridge variant of the
same step, and the CPU oracle timed on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from workloads import ASIAN_LARGE, BASE, QMC_REPLICATES  # noqa: E402

METRIC = "path-steps/s incl. Greeks, adjoint vs bump-revalue; p50/p99 request latency"

# Vector-ALU operations per path-step of the dominant kernel (FP32, Philox,
# Asian with a fixing every step, fused bumps = 5 path states, full
# truncation), counted from the method's arithmetic, one per elementary
# operation (FMA, transcendental, 32x32->64 multiply, XOR, compare/select and
# conversion each count 1): Philox half block 30, two uniforms 6, Box-Muller 7,
# correlation and shared Milstein terms 7, five state updates 5 x 10, fixing
# sums 10 + 4 x 3.  Derivation in the design doc.
OPS_PER_PATH_STEP = 122.0
# Published FP32 vector peak 157.3 TFLOP/s = 78.6e12 FMA lane-operations/s
# (256 CUs x 128 lanes/clk x 2.4 GHz); every counted operation is priced as one
# such lane-operation.
ALU_PEAK_OPS = 256 * 128 * 2.4e9


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU-baseline leg")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    return ap.parse_args()


def cpu_threads() -> int:
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(n, 16))


def cpu_baseline(target_s: float):
    """The oracle (FP64, full re-simulation of each of the 9 scenarios) on a
    bounded prefix of the same workload's paths, scaled to path-steps/s."""
    import oracle
    wl = ASIAN_LARGE
    p = oracle.Params(**wl.params)
    threads = cpu_threads()
    pilot = 2048
    t0 = time.perf_counter()
    oracle.price_greeks(p, wl.opt_type, pilot, wl.n_steps, wl.seed, threads=threads)
    dt = time.perf_counter() - t0
    n = int(min(wl.n_paths, max(pilot, pilot * target_s / max(dt, 1e-6))))
    t0 = time.perf_counter()
    oracle.price_greeks(p, wl.opt_type, n, wl.n_steps, wl.seed, threads=threads)
    dt = time.perf_counter() - t0
    return {"value": n * wl.n_steps / dt, "unit": "path-steps/s", "cores": threads,
            "kind": "oracle",
            "sample": f"first {n} of {wl.n_paths} paths x {wl.n_steps} steps, 9 scenarios "
                      f"re-simulated in FP64 ({dt:.1f} s)"}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU; --gpus {args.gpus} is not supported "
              "(the path shards by path index, see DESIGN.md)", file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_2309_10477_amd as hm

    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        sys.exit(1)
    hm.lib()
    wl = ASIAN_LARGE
    ctx = hm.Context(0)
    opts = hm.Options(precision=hm.FP32)

    def step():
        return ctx.price_greeks(wl.params, wl.opt_type, wl.n_paths, wl.n_steps, wl.seed, opts)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    kernel_ms = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        r = step()
        kernel_ms.append(r["device_ms"])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_per_step = wall / args.steps * 1e3
    path_steps = wl.n_paths * wl.n_steps
    value = path_steps / (wall / args.steps)

    k_ms = float(np.mean(kernel_ms))
    achieved = OPS_PER_PATH_STEP * path_steps / (k_ms * 1e-3)
    roofline = {"bound": "alu", "achieved": achieved / 1e12, "peak": ALU_PEAK_OPS / 1e12,
                "unit": "Top/s", "frac": achieved / ALU_PEAK_OPS, "traffic": None,
                "kernel": "price_kernel<float, Philox, Asian, fused bumps, full truncation>",
                "kernel_ms": k_ms}

    # the same step with Sobol + Brownian-bridge normals (16 shifted replicates)
    qopts = hm.Options(precision=hm.FP32, rng=hm.SOBOL_BRIDGE, qmc_replicates=QMC_REPLICATES)
    for _ in range(2):
        ctx.price_greeks(wl.params, wl.opt_type, wl.n_paths, wl.n_steps, wl.seed, qopts)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    qk = []
    for _ in range(5):
        rq = ctx.price_greeks(wl.params, wl.opt_type, wl.n_paths, wl.n_steps, wl.seed, qopts)
        qk.append(rq["device_ms"])
    torch.cuda.synchronize()
    q_ms = (time.perf_counter() - t1) / 5 * 1e3

    out = {
        "metric": METRIC, "value": value, "unit": "path-steps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": wl.name, "option": "asian_call_daily_fixings",
                   "n_paths": wl.n_paths, "n_steps": wl.n_steps, "rng": "philox4x32-10",
                   "greeks": "price, pathwise delta/rho, bump delta/gamma/vega/rho/theta",
                   "params": BASE},
        "roofline": roofline,
        "estimates": {k: r[k] for k in ("price", "delta", "gamma", "vega", "rho", "theta",
                                        "pw_delta", "pw_rho")},
        "qmc_sobol_bridge": {"value": path_steps / (q_ms * 1e-3), "unit": "path-steps/s",
                             "ms_per_step": q_ms, "kernel_ms": float(np.mean(qk)),
                             "price": rq["price"], "replicates": QMC_REPLICATES},
    }
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(args.cpu_seconds)
    ctx.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
