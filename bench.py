"""Benchmark: path-steps/s with Greeks of the Heston/Milstein Monte-Carlo path on one MI355X.

One step = one pass of the whole path over one batch: the arithmetic-average
Asian call (daily fixings), 2^20 paths x 252 Milstein steps, FP32 path state
with FP64 cross-path sums, Philox normals, price + pathwise Delta/Rho + five
central bump Greeks (Delta, Gamma, Vega, Rho, Theta) on common random numbers,
all estimators reduced across paths and copied to the host.  Inputs are
parameters only (nothing to stage); the timed region covers the library call.

Prints ONE JSON line (rank 0).  Also reported: the roofline of the path kernel
(algorithmic FP32 FLOP per path-step against the FP32 vector peak, with the
VALU utilisation of a counter pass), the latency of the small FP64 European
call, the Sobol + Brownian-bridge variant of the same step, the same step
under the quadratic-exponential scheme, the same step with the
geometric-average control variate, exact (Broadie-Kaya) simulation, the
adjoint against plain bump-and-revalue, the 4096-option batch, the serving
loop's latency, and the CPU oracle timed on bounded samples of the workloads.
"""
from __future__ import annotations

import argparse
import gc
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# HIP maps a process's streams onto GPU_MAX_HW_QUEUES hardware queues (4 by
# default) and streams that share one run one after the other.  The serving
# engine overlaps launches on three streams of its own beside the context's
# (and the control variate's side stream), so this process asks for eight;
# set before anything initialises HIP.
if int(os.environ.get("GPU_MAX_HW_QUEUES", "4")) < 8:
    os.environ["GPU_MAX_HW_QUEUES"] = "8"

from workloads import ASIAN_LARGE, BASE, QMC_REPLICATES  # noqa: E402

METRIC = "path-steps/s incl. Greeks, adjoint vs bump-revalue; p50/p99 request latency"

# Algorithmic FP32 work per path-step of the dominant kernel (Philox, Asian
# with a fixing every step, fused bumps = five path states: base, v0 +/-,
# T +/-; full truncation), on the per-part basis of the method's operation
# count, FMA = 2 FLOP, a transcendental = 1: shared by the five states, two
# uniforms 4, Box-Muller 3 and the correlation 3; per state, the log-price
# step 6, the variance step 9 and the daily fixing 7.  The S0 and r scenarios
# are evaluated from the base state and add no per-step work.
FLOP_PER_PATH_STEP = 10 + 5 * 22
# Published FP32 vector peak of the MI355X: 256 CUs x 2.4 GHz x 256 FLOP per
# clock (packed FP32 FMA).
FP32_VECTOR_PEAK = 157.3e12
# HBM bytes per launch of the path kernel from the FETCH_SIZE / WRITE_SIZE
# counter passes (FETCH_SIZE scaled by 2.00 and WRITE_SIZE by 1.00, the factors
# a 256 MiB device copy reads under the same counters); see
# profiles/price_kernel_asian_2p20x252_fp32_bumps_hbm_counters.md.  Set to None
# whenever the kernel changes until the counters are taken again.
TRAFFIC_BYTES_PER_LAUNCH = 838_265
# VALU utilisation of the path kernel from SQ counter passes of the same
# build: the fraction of SIMD quad-cycles that issue a VALU instruction, the
# share of lanes active in them, and the FLOP the hardware counted; see
# profiles/valu_utilisation_counters.md.  Set to None whenever the kernel
# changes until the counters are taken again.
VALU_COUNTERS = {
    "simd_valu_busy": 0.948,        # (SQ_ACTIVE_INST_VALU - SQ_ACTIVE_INST_VALU2) / SIMD quad-cycles
    "valu_lane_util": 0.9994,       # SQ_THREAD_CYCLES_VALU / (SQ_ACTIVE_INST_VALU x 64)
    "valu_utilisation": 0.947,      # their product: the path kernel's share of VALU issue capacity
    "valubusy_amd_formula": 1.188,  # VALUBusy as rocprof defines it (counts dual-issued quad-cycles twice)
    "counted_flop_per_path_step": 112.9,  # 64 x (SQ_INSTS_VALU_FLOPS_FP32 + _TRANS + FP64 + _TRANS) / path-steps
}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU-baseline leg")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--legs", default="c1,qmc,qe,cv,exact,adjoint,batch,serve",
                    help="extra legs reported after the timed steps: c1, qmc, qe, cv, exact, adjoint, "
                         "batch, serve, "
                         "and copy (a 256 MiB device copy that calibrates HBM byte counters)")
    return ap.parse_args()


def cpu_threads() -> int:
    """Host threads for the oracle: the process's affinity set, bounded by the
    CPU share the launcher grants (OMP_NUM_THREADS, when set)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    share = os.environ.get("OMP_NUM_THREADS", "")
    if share.isdigit() and int(share) > 0:
        n = min(n, int(share))
    return max(1, n)


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


def cpu_oracle_legs():
    """The oracle timed on the other workloads, each on a bounded sample:
    the 1e4 x 100 FP64 European call with its 9 bump scenarios in full; a
    64-option subsample of the 4096-option portfolio (every 64th option, its
    first 2048 paths); the finite-difference reference of the seven adjoint
    sensitivities (15 revaluations) on the first 2^16 paths of the 2^22 x 365
    European call.  Rates are base-scenario path-steps per second."""
    import oracle
    from workloads import ADJOINT_LARGE, EURO_SMALL, portfolio
    threads = cpu_threads()
    out = {"cores": threads, "kind": "oracle"}
    wl = EURO_SMALL
    p = oracle.Params(**wl.params)
    t0 = time.perf_counter()
    oracle.price_greeks(p, wl.opt_type, wl.n_paths, wl.n_steps, wl.seed, threads=threads)
    dt = time.perf_counter() - t0
    out["euro_call_1e4x100_fp64_bumps"] = {"latency_ms": dt * 1e3,
                                           "path_steps_per_s": wl.n_paths * wl.n_steps / dt}
    pf = portfolio()
    idx = np.arange(0, len(pf), 64)
    ps = 0
    t0 = time.perf_counter()
    for i in idx:
        n = int(min(2048, pf.n_paths[i]))
        oracle.simulate(oracle.Params(**pf.params(i)), int(pf.opt_type[i]), int(pf.n_steps[i]),
                        int(pf.seed[i]), 0, n, threads=threads)
        ps += n * int(pf.n_steps[i])
    dt = time.perf_counter() - t0
    out["portfolio_64_option_subsample"] = {
        "path_steps_per_s": ps / dt, "path_steps": ps,
        "extrapolated_portfolio_s": pf.path_steps() / (ps / dt),
        "sample": f"options {idx[0]}, {idx[1]}, ..., {idx[-1]}: first min(2048, n) paths each"}
    A = ADJOINT_LARGE
    p = oracle.Params(**A["params"])
    n, N = 1 << 16, A["n_steps"]
    t0 = time.perf_counter()
    oracle.simulate(p, 0, N, A["seed"], 0, n, threads=threads)
    for name, _, rel, h in ADJ_BUMPS:
        d = h * abs(getattr(p, name)) if rel else h
        for sgn in (1.0, -1.0):
            oracle.simulate(p.replace(**{name: getattr(p, name) + sgn * d}), 0, N, A["seed"], 0,
                            n, threads=threads)
    dt = time.perf_counter() - t0
    out["adjoint_fd_reference_2p16x365"] = {
        "path_steps_per_s": n * N / dt, "seconds": dt,
        "sample": f"first {n} of {A['n_paths']} paths, 15 revaluations"}
    return out


def c1_latency(ctx, hm, torch, reps=200):
    """The 1e4-path x 100-step FP64 European call with price, pathwise Delta/Rho
    and the five central bump Greeks (fused kernel): p50/p99 latency of the
    synchronous library call, results on the host."""
    from workloads import EURO_SMALL as wl
    opts = hm.Options(precision=hm.FP64)
    for _ in range(10):
        ctx.price_greeks(wl.params, wl.opt_type, wl.n_paths, wl.n_steps, wl.seed, opts)
    torch.cuda.synchronize()
    lat, dev = [], []
    for _ in range(reps):
        t0 = time.perf_counter()
        r = ctx.price_greeks(wl.params, wl.opt_type, wl.n_paths, wl.n_steps, wl.seed, opts)
        lat.append((time.perf_counter() - t0) * 1e3)
        dev.append(r["device_ms"])
    lat = np.array(lat)
    return {"workload": wl.name, "calls": reps, "p50_ms": float(np.percentile(lat, 50)),
            "p99_ms": float(np.percentile(lat, 99)), "mean_ms": float(lat.mean()),
            "kernel_ms_mean": float(np.mean(dev)),
            "path_steps_per_s_at_p50": wl.n_paths * wl.n_steps / (np.percentile(lat, 50) * 1e-3),
            "price": r["price"], "delta": r["delta"]}


ADJ_BUMPS = (("S0", 0, 1, 0.01), ("v0", 4, 1, 0.01), ("r", 2, 0, 1e-4), ("kappa", 5, 1, 0.01),
             ("theta", 6, 1, 0.01), ("sigma", 7, 1, 0.01), ("rho", 8, 0, 0.01))


def exact_simulation(ctx, hm, torch):
    """Exact (Broadie-Kaya) simulation, FP64: the European call in one step and
    the paper's quarterly Asian call (paper parameters, four steps), 2^20 paths
    each; price against the characteristic-function price (European)."""
    from workloads import PAPER
    out = {}
    opts = hm.Options(scheme=hm.EXACT, greeks=hm.GREEKS_PATHWISE)
    for name, params, opt, N in (("euro_call_1_step", BASE, hm.EURO_CALL, 1),
                                 ("paper_asian_call_4_steps", PAPER, hm.ASIAN_CALL, 4)):
        n = 1 << 20
        ctx.price_greeks(params, opt, 1 << 16, N, 1, opts)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = ctx.price_greeks(params, opt, n, N, 42, opts)
        wall = time.perf_counter() - t0
        out[name] = {"paths_per_s": n / wall, "path_steps_per_s": n * N / wall,
                     "ms": wall * 1e3, "kernel_ms": r["device_ms"], "price": r["price"]}
    return out


def adjoint_vs_bump(ctx, hm, torch):
    """European and Asian call, 2^22 paths x 365 steps, FP32: the seven
    sensitivities by the adjoint (forward with checkpoints every 16 steps +
    reverse sweep) against plain central bump-and-revalue (15 independent
    revaluations on common random numbers).  speedup_at_equal_se =
    (t_bump / t_adjoint) x (se_bump / se_adjoint)^2 per sensitivity."""
    from workloads import ADJOINT_LARGE as A
    n, N, seed = A["n_paths"], A["n_steps"], A["seed"]
    every = A["checkpoint_every"]
    opts = hm.Options(precision=hm.FP32, greeks=hm.GREEKS_PATHWISE)
    ck = torch.empty(hm.ckpt_bytes(n, N, every, hm.FP32), dtype=torch.uint8, device="cuda:0")
    out = {"n_paths": n, "n_steps": N, "checkpoint_every": every}
    for name, typ in (("euro_call", hm.EURO_CALL), ("asian_call", hm.ASIAN_CALL)):
        for _ in range(2):
            ctx.adjoint_forward(A["params"], typ, n, N, seed, ck, every, opts)
            ctx.adjoint_backward(A["params"], typ, n, N, seed, ck, every, 1.0, opts)
        torch.cuda.synchronize()
        reps = 3
        t0 = time.perf_counter()
        for _ in range(reps):
            price, fms = ctx.adjoint_forward(A["params"], typ, n, N, seed, ck, every, opts)
            grads, bms = ctx.adjoint_backward(A["params"], typ, n, N, seed, ck, every, 1.0, opts)
        torch.cuda.synchronize()
        t_adj = (time.perf_counter() - t0) / reps
        bumps = [(idx, rel, h) for _, idx, rel, h in ADJ_BUMPS]
        ctx.bump_revalue(A["params"], typ, n, N, seed, bumps, opts)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            rb = ctx.bump_revalue(A["params"], typ, n, N, seed, bumps, opts)
        torch.cuda.synchronize()
        t_bump = (time.perf_counter() - t0) / reps
        per = {}
        for k, (pname, _, _, _) in enumerate(ADJ_BUMPS):
            ga, sa = grads[k]
            gb, sb = rb["first"][k]
            per[pname] = {"adjoint": [ga, sa], "bump": [gb, sb],
                          "speedup_at_equal_se": (t_bump / t_adj) * (sb / sa) ** 2}
        out[name] = {
            "price": price, "adjoint_ms": t_adj * 1e3, "forward_kernel_ms": fms,
            "backward_kernel_ms": bms, "bump_ms": t_bump * 1e3,
            "bump_kernels_ms": rb["device_ms"],
            "adjoint_path_steps_per_s": n * N / t_adj,
            "bump_path_steps_per_s": n * N / t_bump,
            "speedup": t_bump / t_adj,
            "min_speedup_at_equal_se": min(v["speedup_at_equal_se"] for v in per.values()),
            "per_parameter": per}
    return out


def portfolio_batch(ctx, hm, torch):
    """The 4096-option portfolio (European/Asian calls and puts, K ~ U[70,130],
    T ~ U[0.1,5], steps = ceil(252 T), paths 2^14..2^20, Heston parameters per
    option) in one persistent launch, FP32 paths, FP64 sums, price + pathwise
    Delta/Rho."""
    from workloads import portfolio
    pf = portfolio()
    reqs = [dict(params=pf.params(i), type=int(pf.opt_type[i]), n_steps=int(pf.n_steps[i]),
                 n_paths=int(pf.n_paths[i]), seed=int(pf.seed[i]), want=hm.WANT_PATHWISE)
            for i in range(len(pf))]
    opts = hm.Options(precision=hm.FP32, greeks=hm.GREEKS_PATHWISE)
    ctx.price_batch(reqs[:64], opts)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res, ms = ctx.price_batch(reqs, opts)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ps = pf.path_steps()
    return {"options": len(pf), "path_steps": ps, "wall_ms": wall * 1e3, "kernel_ms": ms,
            "path_steps_per_s": ps / wall, "kernel_path_steps_per_s": ps / (ms * 1e-3)}


def variant_steps(ctx, torch, wl, opts, warmup=20, reps=30):
    """The timed step's workload under other options: `warmup` untimed calls
    (the clocks settle over some tens of milliseconds after a change of
    kernel), then `reps` timed calls.  Returns (last result, wall ms per call,
    [path-kernel ms per call])."""
    for _ in range(warmup):
        ctx.price_greeks(wl.params, wl.opt_type, wl.n_paths, wl.n_steps, wl.seed, opts)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ks = []
    for _ in range(reps):
        r = ctx.price_greeks(wl.params, wl.opt_type, wl.n_paths, wl.n_steps, wl.seed, opts)
        ks.append(r["device_ms"])
    torch.cuda.synchronize()
    return r, (time.perf_counter() - t1) / reps * 1e3, ks


def serving(ctx, hm, torch, n_measured=2000, n_warm=100):
    """Continuous batching: requests (50/50 European/Asian, calls/puts, path cap
    2^U[12,22], steps U{50..1000}, Heston parameters as the portfolio's, price
    + seven adjoint sensitivities to a price SE of 0.1).  Saturation: after an
    untimed burst of n_measured other requests on the same server, n_measured
    requests submitted at once (built beforehand); its rate is the completed
    work over the time from the first submission to the last completion (as
    the server timed it), drain included.  Then, still on that server (a
    serving engine runs warm), Poisson streams at 0.5 and 0.8 of the saturated
    request rate, n_warm + n_measured requests each, latency (heston_submit to
    completion) of the last n_measured.  Path-steps count the paths each
    result uses (whole 1024-path items up to the one that met the target); the
    scheduled figure adds the items computed past it."""
    from workloads import request_stream

    def to_reqs(rs):
        return [dict(params=rs.params[i], type=int(rs.opt_type[i]), n_steps=int(rs.n_steps[i]),
                     n_paths=int(rs.path_cap[i]), seed=int(rs.seed[i]), want=hm.WANT_ADJOINT,
                     se_target=rs.se_target) for i in range(len(rs.params))]

    def run(srv, reqs, arrivals):
        # The run ends at the last completion as the server saw it (each
        # request's submission time plus its latency), so that a pause of this
        # client while it collects results does not count; the cyclic garbage
        # collector stays off meanwhile, so it cannot delay submissions.
        built = [hm.make_request(**q) for q in reqs]
        st0 = srv.stats()
        gc.collect()
        gc.disable()
        try:
            t0 = time.perf_counter()
            tickets, t_sub = [], []
            for c, a in zip(built, arrivals):
                while time.perf_counter() - t0 < a:
                    pass
                t_sub.append(time.perf_counter() - t0)
                tickets.append(srv.submit_request(c))
            res = [srv.wait(t, 300_000) for t in tickets]
        finally:
            gc.enable()
        wall = max(ts + r["latency_ms"] * 1e-3 for ts, r in zip(t_sub, res))
        st = {k: v - st0[k] for k, v in srv.stats().items()}
        return res, wall, st

    def useful(reqs, res):
        # path-steps behind the results: each request's paths used x its steps
        return float(sum(r["n_paths"] * q["n_steps"] for q, r in zip(reqs, res)))

    def load_record(rate, reqs, res, wall, st):
        # latency of the last n_measured requests; rates over the whole stream
        lat = np.array([r["latency_ms"] for r in res[n_warm:]])
        return {"arrival_rate_per_s": rate, "requests": n_measured,
                "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
                "mean_ms": float(lat.mean()), "throughput_requests_per_s": len(res) / wall,
                "path_steps_per_s": useful(reqs, res) / wall,
                "scheduled_path_steps_per_s": st["path_steps"] / wall,
                "launches": st["launches"], "gpu_busy_frac": st["busy_ms"] * 1e-3 / wall}

    srv = hm.Server(ctx, precision=hm.FP32, max_steps=1000)
    try:
        # the first burst in a process runs 10-15% slower than later ones (the
        # runtime's pools grow over it), so the untimed warm-up burst has the
        # measured burst's size
        warm = to_reqs(request_stream(n_measured, 1.0, seed=4))
        run(srv, warm, np.zeros(n_measured))
        burst = to_reqs(request_stream(n_measured, 1.0, seed=5))
        res, wall, st = run(srv, burst, np.zeros(n_measured))
        mu = n_measured / wall
        out = {"saturated_requests": n_measured, "saturated_requests_per_s": mu,
               "saturated_path_steps_per_s": useful(burst, res) / wall,
               "saturated_scheduled_path_steps_per_s": st["path_steps"] / wall,
               "saturated_gpu_busy_frac": st["busy_ms"] * 1e-3 / wall,
               "mean_paths_used": float(np.mean([r["n_paths"] for r in res]))}
        for frac in (0.5, 0.8):
            rs = request_stream(n_warm + n_measured, frac * mu, seed=6)
            reqs = to_reqs(rs)
            res, wall, st = run(srv, reqs, rs.arrival_s)
            out[f"load_{frac}"] = load_record(frac * mu, reqs, res, wall, st)
    finally:
        srv.close()
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: runs on one GPU; --gpus {args.gpus} is not supported "
              "(paths would shard across GPUs by path index, with one all-reduce of the "
              "FP64 partial sums)", file=sys.stderr)
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
    achieved = FLOP_PER_PATH_STEP * path_steps / (k_ms * 1e-3)
    roofline = {"bound": "alu", "achieved": achieved / 1e12, "peak": FP32_VECTOR_PEAK / 1e12,
                "unit": "TFLOP/s", "frac": achieved / FP32_VECTOR_PEAK,
                "traffic": TRAFFIC_BYTES_PER_LAUNCH,
                "basis": f"algorithmic FP32 FLOP, {FLOP_PER_PATH_STEP} per path-step "
                         "(FMA = 2, transcendental = 1), per launch / mean launch time",
                "kernel": "price_kernel<float, Philox, Asian, fused bumps, full truncation>",
                "kernel_ms": k_ms}
    if VALU_COUNTERS is not None:
        roofline["valu_counters"] = VALU_COUNTERS

    legs = set(a for a in args.legs.split(",") if a)
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
    }
    if "c1" in legs:
        out["euro_small_latency"] = c1_latency(ctx, hm, torch)
    if "qmc" in legs:
        # the same step with Sobol + Brownian-bridge normals (16 shifted replicates)
        qopts = hm.Options(precision=hm.FP32, rng=hm.SOBOL_BRIDGE, qmc_replicates=QMC_REPLICATES)
        rq, q_ms, qk = variant_steps(ctx, torch, wl, qopts)
        out["qmc_sobol_bridge"] = {"value": path_steps / (q_ms * 1e-3), "unit": "path-steps/s",
                                   "ms_per_step": q_ms, "kernel_ms": float(np.mean(qk)),
                                   "price": rq["price"], "replicates": QMC_REPLICATES}
    if "qe" in legs:
        # the same step under Andersen's QE scheme (one Philox block per step)
        eopts = hm.Options(precision=hm.FP32, scheme=hm.QE)
        re_, e_ms, ek = variant_steps(ctx, torch, wl, eopts)
        out["qe_scheme"] = {"value": path_steps / (e_ms * 1e-3), "unit": "path-steps/s",
                            "ms_per_step": e_ms, "kernel_ms": float(np.mean(ek)),
                            "price": re_["price"]}
    if "cv" in legs:
        # the same step with the geometric-average control variate on the price:
        # wall time includes the control's device-side transform price
        copts = hm.Options(precision=hm.FP32, control_variate=hm.CONTROL_GEOMETRIC)
        rc, c_ms, ck = variant_steps(ctx, torch, wl, copts)
        vrf = (rc["price"][1] / rc["cv_price"][1]) ** 2
        out["geometric_control_variate"] = {
            "value": path_steps / (c_ms * 1e-3), "unit": "path-steps/s", "ms_per_step": c_ms,
            "kernel_ms": float(np.mean(ck)), "price": rc["price"], "cv_price": rc["cv_price"],
            "cv_beta": rc["cv_beta"], "cv_mean": rc["cv_mean"], "variance_reduction": vrf,
            "equal_se_path_steps_per_s": path_steps / (c_ms * 1e-3) * vrf}
    if "exact" in legs:
        out["exact_simulation"] = exact_simulation(ctx, hm, torch)
    if "adjoint" in legs:
        out["adjoint_vs_bump"] = adjoint_vs_bump(ctx, hm, torch)
    if "batch" in legs:
        out["portfolio_batch"] = portfolio_batch(ctx, hm, torch)
    if "serve" in legs:
        out["serving"] = serving(ctx, hm, torch)
    if "copy" in legs:
        src = torch.empty(64 << 20, dtype=torch.float32, device="cuda:0").fill_(1.0)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        out["copy_calibration_bytes"] = src.numel() * 4
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(args.cpu_seconds)
        out["cpu_oracle_legs"] = cpu_oracle_legs()
    ctx.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
