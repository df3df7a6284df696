"""GPU parity: the HIP path against the CPU oracle, through the C ABI.

Per path (heston_dump_paths records, produced by the pricing kernel itself)
against oracle.simulate / oracle.scenario_payoffs on the same seeded stream,
with |gpu - oracle| <= tol * max(|oracle|, floor): floors S0 for prices,
averages and payoffs, max(v0, theta) for the variance, 1 for pathwise Delta,
K T for pathwise Rho; tol = 1e-12 (FP64 kernels) and 1e-5 (FP32 kernels).
A payoff indicator may differ only on paths with |X - K| < 1e3 tol K.
Reduced estimates are checked against the same per-path values summed on the
host.
"""
import math
import os

import numpy as np
import pytest

import oracle
from workloads import BASE, PAPER, paper_fixing_steps

pytestmark = pytest.mark.gpu

PB = oracle.Params(**BASE)
PP = oracle.Params(**PAPER)
TOL = {0: 1e-12, 1: 1e-5}


@pytest.fixture(scope="module")
def hm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2309_10477_amd as hm
    hm.lib()
    return hm


@pytest.fixture(scope="module")
def ctx(hm):
    c = hm.Context(0)
    yield c
    c.close()


def floors(p):
    return {"S_T": p.S0, "V_T": max(p.v0, p.theta, 1e-3), "Sbar": p.S0, "pay": p.S0,
            "pw_delta": 1.0, "pw_rho": p.K * p.T}


def compare(name, g, o, tol, floor, allow=None):
    err = np.abs(g - o) / np.maximum(np.abs(o), floor)
    bad = err > tol
    if allow is not None:
        bad &= ~allow
    if bad.any():
        i = int(np.argmax(np.where(bad, err, 0)))
        raise AssertionError(f"{name}: {int(bad.sum())} paths off, worst path {i}: "
                             f"gpu {g[i]!r} oracle {o[i]!r} rel {err[i]:.3e} > {tol}")


def check_records(dump, p, opt_type, n_steps, seed, first, count, prec, scheme, fixings, bumps,
                  za=None, zb=None, threads=8):
    tol = TOL[prec]
    mode = {0: oracle.FULL_TRUNC, 1: oracle.ABSORB, 3: oracle.EULER_FULL_TRUNC,
            4: oracle.EULER_ABSORB, 5: oracle.PARTIAL_TRUNC, 6: oracle.REFLECT}[scheme]
    rec = oracle.simulate(p, opt_type, n_steps, seed, first, count, mode, fixings, za, zb, threads)
    X = rec[:, 2]
    near = np.abs(X - p.K) < 1e3 * tol * p.K
    fl = floors(p)
    for k, name in enumerate(oracle.REC_FIELDS):
        compare(name, dump[:, k], rec[:, k], tol, fl[name],
                allow=near if name in ("pw_delta", "pw_rho") else None)
    compare("x_T", dump[:, 14], np.log(rec[:, 0] / p.S0), tol, 1.0)
    if bumps:
        pay, _ = oracle.scenario_payoffs(p, opt_type, n_steps, seed, count, first, mode, fixings,
                                         za=za, zb=zb, threads=threads)
        for k, sc in enumerate(oracle.SCENARIOS[1:]):
            # payoffs are continuous in the average, so no indicator allowance
            compare("pay_" + sc, dump[:, 6 + k], pay[sc], tol, p.S0)
    else:
        assert np.isnan(dump[:, 6:14]).all()
    return rec


def dump(hm, ctx, p, opt_type, n_paths, n_steps, seed, first, count, opts):
    t = ctx.dump_paths(p.__dict__, opt_type, n_paths, n_steps, seed, first, count, opts)
    return t.cpu().numpy()


# ---------------------------------------------------------------------------

def test_european_fp64_bumps_full_parity(hm, ctx):
    """European call, 1e4 paths x 100 steps, FP64, bumps on common random
    numbers: every path, every scenario."""
    n, N, seed = 10_000, 100, 42
    opts = hm.Options()
    d = dump(hm, ctx, PB, hm.EURO_CALL, n, N, seed, 0, n, opts)
    check_records(d, PB, oracle.EURO_CALL, N, seed, 0, n, 0, 0, None, True)
    r = ctx.price_greeks(PB.__dict__, hm.EURO_CALL, n, N, seed, opts)
    ref = oracle.price_greeks(PB, oracle.EURO_CALL, n, N, seed, threads=8)
    for k, (v, se) in ref.items():
        assert r[k][0] == pytest.approx(v, rel=1e-10, abs=1e-12), k
        assert r[k][1] == pytest.approx(se, rel=1e-6), k


@pytest.mark.parametrize("opt_type", [0, 1, 2, 3])
@pytest.mark.parametrize("scheme", [0, 1, 3, 4, 5, 6])
def test_fp64_all_types_ragged(hm, ctx, opt_type, scheme):
    """Milstein (0, 1) and the paper's Euler discretisation (3, 4), each under
    full truncation and absorption; Milstein with partial truncation (5) and
    reflection (6), at a vol of vol that often turns the variance negative."""
    n, N, seed = 1000 + 37, 7, 0xDEADBEEF12345
    fix = (2, 3, 7) if opt_type >= 2 else None
    p = PP if scheme in (1, 4) else PB
    if scheme in (5, 6):
        p = PB.replace(v0=0.01, sigma=1.0, kappa=1.0, theta=0.02)
    opts = hm.Options(scheme=scheme, fixings=fix)
    d = dump(hm, ctx, p, opt_type, n, N, seed, 0, n, opts)
    check_records(d, p, opt_type, N, seed, 0, n, 0, scheme, fix, True)


def _estimates_match(r, ref):
    # Where a Greek's samples vanish on every path (a Gamma over a few paths
    # all on one side of the strike) its standard error is rounding noise, so
    # the error takes the estimate's absolute floor.
    for k, (v, se) in ref.items():
        assert r[k][0] == pytest.approx(v, rel=1e-10, abs=1e-12), k
        assert r[k][1] == pytest.approx(se, rel=1e-6, abs=1e-12), k


@pytest.mark.parametrize("opt_type", [0, 1, 2, 3])
@pytest.mark.parametrize("scheme", [0, 1, 3, 4])
@pytest.mark.parametrize("n", [5, 1037])
def test_fp64_small_bump_estimates(hm, ctx, opt_type, scheme, n):
    """Estimates of small FP64 bump launches, which the kernel lays out one
    scenario per lane: a count below one wave's paths and a ragged count over
    many blocks, Milstein and Euler under both fixes, daily and sparse
    fixings."""
    N, seed = 11, 0x5EED0000 + n
    fix = (1, 4, 11) if opt_type >= 2 else None
    p = PP if scheme in (1, 4) else PB
    mode = {0: oracle.FULL_TRUNC, 1: oracle.ABSORB, 3: oracle.EULER_FULL_TRUNC,
            4: oracle.EULER_ABSORB}[scheme]
    r = ctx.price_greeks(p.__dict__, opt_type, n, N, seed, hm.Options(scheme=scheme, fixings=fix))
    ref = oracle.price_greeks(p, opt_type, n, N, seed, mode, fix, threads=8)
    _estimates_match(r, ref)


@pytest.mark.parametrize("prec,h", [(0, 1e-3), (1, 3e-3)])
def test_fused_r_bump_at_its_largest(hm, ctx, prec, h):
    """The largest r bump the fused arithmetic-Asian kernel takes (bump_r_abs T
    = 1e-3 in FP64, 3e-3 in FP32), where its Taylor series of e^{+-h t} over
    the fixings is least accurate: per-path r-bumped payoffs against the
    oracle's, which bumps r exactly, and in FP64 the estimates."""
    n, N, seed = 1037, 12, 99
    opts = hm.Options(precision=prec, bump_r_abs=h)
    d = dump(hm, ctx, PB, hm.ASIAN_CALL, n, N, seed, 0, n, opts)
    bumps = oracle.Bumps(r_abs=h)
    pay, _ = oracle.scenario_payoffs(PB, oracle.ASIAN_CALL, N, seed, n, 0, oracle.FULL_TRUNC,
                                     None, bumps, threads=8)
    for k, sc in enumerate(oracle.SCENARIOS[1:]):
        if sc in ("r+", "r-"):
            compare("pay_" + sc, d[:, 6 + k], pay[sc], TOL[prec], PB.S0)
    if prec == 0:
        r = ctx.price_greeks(PB.__dict__, hm.ASIAN_CALL, n, N, seed, opts)
        _estimates_match(r, oracle.price_greeks(PB, oracle.ASIAN_CALL, n, N, seed,
                                                bumps=bumps, threads=8))


@pytest.mark.parametrize("opt_type,n", [(0, 36864), (0, 36865), (3, 98304), (3, 98305)])
def test_fp64_bump_estimates_at_layout_limit(hm, ctx, opt_type, n):
    """Either side of the largest count laid out one scenario per lane
    (36864 European, 98304 Asian paths): both layouts give the oracle's
    estimates."""
    N, seed = 9, 77
    r = ctx.price_greeks(PB.__dict__, opt_type, n, N, seed, hm.Options())
    _estimates_match(r, oracle.price_greeks(PB, opt_type, n, N, seed, threads=8))


@pytest.mark.parametrize("opt_type", [0, 1, 2, 3])
def test_fp32_all_types(hm, ctx, opt_type):
    n, N, seed = 4096 + 100, 63, 7
    opts = hm.Options(precision=hm.FP32)
    d = dump(hm, ctx, PB, opt_type, n, N, seed, 0, n, opts)
    check_records(d, PB, opt_type, N, seed, 0, n, 1, 0, None, True)


@pytest.mark.parametrize("scheme", [3, 4, 5, 6])
def test_euler_and_fixes_fp32(hm, ctx, scheme):
    n, N, seed = 4096 + 100, 63, 9
    opts = hm.Options(precision=hm.FP32, scheme=scheme)
    d = dump(hm, ctx, PB, hm.ASIAN_PUT, n, N, seed, 0, n, opts)
    check_records(d, PB, oracle.ASIAN_PUT, N, seed, 0, n, 1, scheme, None, True)


@pytest.mark.parametrize("scheme", [3, 6])
def test_non_milstein_truncations_rejected_by_adjoint_and_batch(hm, ctx, scheme):
    import torch
    opts = hm.Options(precision=hm.FP32, scheme=scheme)
    ck = torch.empty(hm.ckpt_bytes(256, 8, 8, hm.FP32), dtype=torch.uint8, device="cuda:0")
    with pytest.raises(hm.HestonError) as e:
        ctx.adjoint_forward(PB.__dict__, 0, 256, 8, 1, ck, 8, opts)
    assert e.value.status == -5
    with pytest.raises(hm.HestonError) as e:
        ctx.price_batch([dict(params=PB.__dict__, type=0, n_steps=4, n_paths=100, seed=1, want=1)],
                        opts)
    assert e.value.status == -5


def test_asian_fp32_daily_fixings_252_steps(hm, ctx):
    n, N, seed = 1 << 14, 252, 42
    opts = hm.Options(precision=hm.FP32)
    d = dump(hm, ctx, PB, hm.ASIAN_CALL, n, N, seed, 0, n, opts)
    check_records(d, PB, oracle.ASIAN_CALL, N, seed, 0, n, 1, 0, None, True)


def test_paper_quarterly_asian_absorption(hm, ctx):
    N = 128
    fix = paper_fixing_steps(N)
    opts = hm.Options(scheme=hm.ABSORPTION, fixings=fix)
    d = dump(hm, ctx, PP, hm.ASIAN_CALL, 3000, N, 1, 0, 3000, opts)
    check_records(d, PP, oracle.ASIAN_CALL, N, 1, 0, 3000, 0, 1, fix, True)


def test_asian_fp32_large_sampled_and_reduction(hm, ctx):
    """The 2^20-path x 252-step FP32 Asian call with five bump Greeks, in the
    launch the benchmark times: sampled paths against the oracle, and the
    reduced estimates against the host sum of every path's record."""
    n, N, seed = 1 << 20, 252, 42
    opts = hm.Options(precision=hm.FP32)
    r = ctx.price_greeks(PB.__dict__, hm.ASIAN_CALL, n, N, seed, opts)
    full = dump(hm, ctx, PB, hm.ASIAN_CALL, n, N, seed, 0, n, opts)
    for first in (0, n // 2 + 12345, n - 700):
        check_records(full[first:first + 700], PB, oracle.ASIAN_CALL, N, seed, first, 700, 1, 0,
                      None, True)
    pay = {sc: full[:, 6 + k] for k, sc in enumerate(oracle.SCENARIOS[1:])}
    pay["base"] = full[:, 3]
    samples = oracle.greek_samples(pay, PB)
    samples["pw_delta"], samples["pw_rho"] = full[:, 4], full[:, 5]
    for k, y in samples.items():
        m, se = oracle.mean_se(y)
        assert r[k][0] == pytest.approx(m, rel=1e-9, abs=1e-12), k
        assert r[k][1] == pytest.approx(se, rel=1e-6), k


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("N", [1, 5, 64])
def test_sobol_bridge_parity(hm, ctx, prec, N):
    from oracle import sobol
    R, M, seed = 4, 700, 42
    n = R * M
    opts = hm.Options(precision=prec, rng=hm.SOBOL_BRIDGE, qmc_replicates=R)
    d = dump(hm, ctx, PB, hm.ASIAN_CALL, n, N, seed, 0, n, opts)
    za, zb = sobol.normals(N, 0, n, R, M, seed)
    check_records(d, PB, oracle.ASIAN_CALL, N, seed, 0, n, prec, 0, None, True, za, zb)
    r = ctx.price_greeks(PB.__dict__, hm.ASIAN_CALL, n, N, seed, opts)
    means = d[:, 3].reshape(R, M).mean(axis=1)
    assert r["price"][0] == pytest.approx(means.mean(), rel=1e-12)
    assert r["price"][1] == pytest.approx(means.std(ddof=1) / math.sqrt(R), rel=1e-9)


def test_sobol_bridge_full_size_sampled(hm, ctx):
    from oracle import sobol
    R, M, N, seed = 16, 1 << 16, 252, 42
    n = R * M
    opts = hm.Options(precision=hm.FP32, rng=hm.SOBOL_BRIDGE, qmc_replicates=R)
    # first = 0 and 3M + 64 * 1001 are 64-point aligned (per-block high-part
    # table; block 1001 has five Gray-code bits >= 6 set), the others are not
    for first in (0, 3 * M + 64 * 1001, 5 * M - 300, n - 500):
        d = dump(hm, ctx, PB, hm.ASIAN_CALL, n, N, seed, first, 500, opts)
        za, zb = sobol.normals(N, first, 500, R, M, seed)
        check_records(d, PB, oracle.ASIAN_CALL, N, seed, first, 500, 1, 0, None, True, za, zb)


@pytest.mark.parametrize("prec", [0, 1])
def test_sobol_aligned_table_equals_generic_points(hm, ctx, prec):
    """Launches whose waves start on 64-point blocks take the high Gray-code
    part of each point from a per-block table; a launch shifted by one path
    combines every direction number itself.  Both give the same records."""
    R, M, N, seed = 2, 1 << 14, 8, 7
    n = R * M
    opts = hm.Options(precision=prec, rng=hm.SOBOL_BRIDGE, qmc_replicates=R)
    a = dump(hm, ctx, PB, hm.ASIAN_PUT, n, N, seed, 0, n, opts)
    b = dump(hm, ctx, PB, hm.ASIAN_PUT, n, N, seed, 1, n - 1, opts)
    np.testing.assert_array_equal(a[1:], b)


def test_path_index_above_2_32_and_wide_seed(hm, ctx):
    first, count, N, seed = (1 << 32) + 5, 300, 9, (7 << 40) | 3
    opts = hm.Options()
    d = dump(hm, ctx, PB, hm.EURO_PUT, first + count, N, seed, first, count, opts)
    check_records(d, PB, oracle.EURO_PUT, N, seed, first, count, 0, 0, None, True)


def test_minimum_paths_and_one_step(hm, ctx):
    r = ctx.price_greeks(PB.__dict__, hm.EURO_CALL, 2, 1, 3, hm.Options())
    rec = oracle.simulate(PB, oracle.EURO_CALL, 1, 3, 0, 2)
    m, se = oracle.mean_se(rec[:, 3])
    assert r["price"][0] == pytest.approx(m, rel=1e-12, abs=1e-13)
    assert r["price"][1] == pytest.approx(se, rel=1e-9, abs=1e-13)


def test_default_entry_point_matches_ex(hm, ctx):
    a = hm.price_greeks(PB.__dict__, hm.EURO_CALL, 10_000, 100, 42)
    b = ctx.price_greeks(PB.__dict__, hm.EURO_CALL, 10_000, 100, 42, hm.Options())
    for k in hm.EST_NAMES:
        assert a[k] == b[k], k


def test_bitwise_reproducible(hm, ctx):
    opts = hm.Options(precision=hm.FP32)
    a = ctx.price_greeks(PB.__dict__, hm.ASIAN_PUT, 100_000, 50, 9, opts)
    b = ctx.price_greeks(PB.__dict__, hm.ASIAN_PUT, 100_000, 50, 9, opts)
    for k in hm.EST_NAMES:
        assert a[k] == b[k], k


def test_statistics_against_analytic(hm, ctx):
    """FP32, 2^20 paths x 100 steps: European call price and Greeks within
    4 SE plus a discretisation allowance of the analytic Heston values."""
    from oracle import analytic
    g = analytic.heston_call_greeks(PB)
    r = ctx.price_greeks(PB.__dict__, hm.EURO_CALL, 1 << 20, 100, 42,
                         hm.Options(precision=hm.FP32))
    bias = {"price": 0.01, "delta": 5e-4, "gamma": 2e-4, "vega": 0.2, "rho": 0.1, "theta": 0.05,
            "pw_delta": 5e-4, "pw_rho": 0.1}
    for k, b in bias.items():
        ref = g[{"pw_delta": "delta", "pw_rho": "rho"}.get(k, k)]
        assert abs(r[k][0] - ref) < 4 * r[k][1] + b, (k, r[k], ref)


@pytest.mark.parametrize("bad", ["nan", "paths", "rho", "fix", "reps", "steps"])
def test_invalid_arguments_are_rejected(hm, ctx, bad):
    p = dict(BASE)
    n, N, opts = 1000, 10, hm.Options()
    if bad == "nan":
        p["sigma"] = float("nan")
    elif bad == "paths":
        n = 1
    elif bad == "rho":
        p["rho"] = 1.5
    elif bad == "fix":
        opts = hm.Options(fixings=(3, 3, 5))
        with pytest.raises(hm.HestonError) as e:
            ctx.price_greeks(p, hm.ASIAN_CALL, n, N, 1, opts)
        assert e.value.status == -1
        return
    elif bad == "reps":
        opts = hm.Options(rng=hm.SOBOL_BRIDGE, qmc_replicates=3)
    elif bad == "steps":
        N = 0
    with pytest.raises(hm.HestonError) as e:
        ctx.price_greeks(p, hm.EURO_CALL, n, N, 1, opts)
    assert e.value.status == -1


# --- geometric averages -----------------------------------------------------

@pytest.mark.parametrize("opt_type", [4, 5])
@pytest.mark.parametrize("scheme", [0, 1, 5])
@pytest.mark.parametrize("fix", [None, (2, 3, 7)], ids=["every-step", "dates"])
def test_geometric_fp64_ragged(hm, ctx, opt_type, scheme, fix):
    n, N, seed = 1000 + 37, 7, 0xDEADBEEF12345
    p = PP if scheme == 1 else PB
    opts = hm.Options(scheme=scheme, fixings=fix)
    d = dump(hm, ctx, p, opt_type, n, N, seed, 0, n, opts)
    check_records(d, p, opt_type, N, seed, 0, n, 0, scheme, fix, True)


@pytest.mark.parametrize("opt_type", [4, 5])
def test_geometric_fp32_daily_fixings(hm, ctx, opt_type):
    n, N, seed = 4096 + 100, 252, 11
    d = dump(hm, ctx, PB, opt_type, n, N, seed, 0, n, hm.Options(precision=hm.FP32))
    check_records(d, PB, opt_type, N, seed, 0, n, 1, 0, None, True)


@pytest.mark.parametrize("prec", [0, 1])
def test_geometric_sobol_bridge(hm, ctx, prec):
    from oracle import sobol
    R, M, N, seed = 4, 700, 12, 5
    n = R * M
    opts = hm.Options(precision=prec, rng=hm.SOBOL_BRIDGE, qmc_replicates=R,
                      fixings=(3, 6, 9, 12))
    d = dump(hm, ctx, PB, hm.GEO_ASIAN_CALL, n, N, seed, 0, n, opts)
    za, zb = sobol.normals(N, 0, n, R, M, seed)
    check_records(d, PB, oracle.GEO_ASIAN_CALL, N, seed, 0, n, prec, 0, (3, 6, 9, 12), True,
                  za, zb)


def test_geometric_estimates_match_oracle(hm, ctx):
    n, N, seed = 20_000, 24, 3
    opts = hm.Options()
    r = ctx.price_greeks(PB.__dict__, hm.GEO_ASIAN_PUT, n, N, seed, opts)
    ref = oracle.price_greeks(PB, oracle.GEO_ASIAN_PUT, n, N, seed, threads=8)
    for k, (v, se) in ref.items():
        assert r[k][0] == pytest.approx(v, rel=1e-10, abs=1e-12), k
        assert r[k][1] == pytest.approx(se, rel=1e-6), k


def test_geometric_price_against_transform(hm, ctx):
    """FP32, 2^22 paths, monthly fixings on a daily grid: the Monte-Carlo price
    sits within 3.5 standard errors, plus the difference to the same dates on a
    grid twice as fine, of the characteristic-function price of the geometric
    average."""
    from oracle import analytic
    N = 252
    steps = tuple(range(21, 253, 21))
    ref = analytic.geometric_asian_call(PB, np.array(steps) / N * PB.T)
    o1 = hm.Options(precision=hm.FP32, fixings=steps)
    o2 = hm.Options(precision=hm.FP32, fixings=tuple(2 * s for s in steps))
    a = ctx.price_greeks(PB.__dict__, hm.GEO_ASIAN_CALL, 1 << 22, N, 17, o1)["price"]
    b = ctx.price_greeks(PB.__dict__, hm.GEO_ASIAN_CALL, 1 << 22, 2 * N, 17, o2)["price"]
    assert abs(a[0] - ref) < 3.5 * a[1] + abs(a[0] - b[0])


def test_geometric_rejected_by_adjoint_and_batch(hm, ctx):
    import torch
    ck = torch.empty(hm.ckpt_bytes(256, 8, 8, hm.FP64), dtype=torch.uint8, device="cuda:0")
    with pytest.raises(hm.HestonError) as e:
        ctx.adjoint_forward(PB.__dict__, hm.GEO_ASIAN_CALL, 256, 8, 1, ck, 8, hm.Options())
    assert e.value.status == -5
    with pytest.raises(hm.HestonError) as e:
        ctx.price_batch([dict(params=PB.__dict__, type=hm.GEO_ASIAN_PUT, n_steps=4, n_paths=100,
                              seed=1, want=1)], hm.Options())
    assert e.value.status == -5


# --- the paper's tables, reproduced on the GPU -------------------------------

def _gold():
    import json
    here = os.path.dirname(os.path.abspath(__file__))
    return json.load(open(os.path.join(here, "golden", "paper_values.json")))


@pytest.mark.parametrize("asian", [False, True], ids=["european", "asian"])
def test_paper_milstein_tables(hm, ctx, asian):
    """The paper's Milstein tables (paper parameters, absorption, 32 000 paths,
    32 to 256 steps; 30-run mean and std): one FP64 run per row within 4
    combined errors, as the oracle's pin."""
    tab = _gold()["milstein_asian_cpu_32000_paths" if asian else
                  "milstein_european_cpu_32000_paths"]
    for N, val, std in zip(tab["steps"], tab["value"], tab["std"]):
        opts = hm.Options(scheme=hm.ABSORPTION, greeks=hm.GREEKS_PATHWISE,
                          fixings=paper_fixing_steps(N) if asian else None)
        r = ctx.price_greeks(PP.__dict__, hm.ASIAN_CALL if asian else hm.EURO_CALL, 32000, N,
                             1000 + N, opts)
        assert abs(r["price"][0] - val) < 4 * math.hypot(r["price"][1], std), (N, r["price"])


def test_paper_greeks_table(hm, ctx):
    """FP32, 2^22 paths, 128 steps, absorption: the European pathwise Delta and
    Rho against the analytic values of the paper's Greeks table (4 SE plus 0.2%
    for the discretisation), the quarterly Asian ones against its
    exact-simulation values (4 SE plus 0.5%: their own error is not printed)."""
    g = _gold()["greeks_table"]
    N = 128
    opts = hm.Options(precision=hm.FP32, scheme=hm.ABSORPTION, greeks=hm.GREEKS_PATHWISE)
    r = ctx.price_greeks(PP.__dict__, hm.EURO_CALL, 1 << 22, N, 7, opts)
    for k, ref in (("pw_delta", g["european"]["delta"]), ("pw_rho", g["european"]["rho"])):
        assert abs(r[k][0] - ref) < 4 * r[k][1] + 0.002 * ref, (k, r[k], ref)
    opts = hm.Options(precision=hm.FP32, scheme=hm.ABSORPTION, greeks=hm.GREEKS_PATHWISE,
                      fixings=paper_fixing_steps(N))
    r = ctx.price_greeks(PP.__dict__, hm.ASIAN_CALL, 1 << 22, N, 8, opts)
    for k, ref in (("pw_delta", g["asian"]["ex_delta"]), ("pw_rho", g["asian"]["ex_rho"])):
        assert abs(r[k][0] - ref) < 4 * r[k][1] + 0.005 * ref, (k, r[k], ref)


@pytest.mark.parametrize("asian", [False, True], ids=["european", "asian"])
def test_paper_path_count_tables(hm, ctx, asian):
    """The paper's path-count tables (paper parameters, absorption, 128 steps,
    4000 to 32 000 paths; 30-run mean and std): one FP64 run per row within 4
    combined errors."""
    tab = _gold()["milstein_asian_paths_128_steps" if asian else
                  "milstein_european_paths_128_steps"]
    N = 128
    opts = hm.Options(scheme=hm.ABSORPTION, greeks=hm.GREEKS_PATHWISE,
                      fixings=paper_fixing_steps(N) if asian else None)
    for n, val, std in zip(tab["paths"], tab["value"], tab["std"]):
        r = ctx.price_greeks(PP.__dict__, hm.ASIAN_CALL if asian else hm.EURO_CALL, n, N,
                             2000 + n, opts)
        assert abs(r["price"][0] - val) < 4 * math.hypot(r["price"][1], std), (n, r["price"])


def test_sobol_directions_wider_than_30_bits_rejected(hm, ctx):
    """The kernels read 30-bit coordinates (the upper half of the unit interval is
    mapped by complementing those 30 bits), so a direction number with bit 30 or
    31 set is an invalid argument; the same table with it cleared is accepted."""
    import ctypes
    N = 8
    o = hm._OptsHolder(hm.Options(rng=hm.SOBOL_BRIDGE, qmc_replicates=2), N)
    dirs = o.dirs.copy()
    dirs[2 * N - 1, 3] |= np.uint32(1 << 30)
    o.dirs = dirs
    o.c.sobol_directions = dirs.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32))
    res = hm.CResult()
    cp = hm._cparams(PB.__dict__)
    st = hm.lib().heston_price_greeks_ex(ctx.handle, ctypes.byref(cp), 0, 512, N, 1,
                                         ctypes.byref(o.c), ctypes.byref(res))
    assert st == -1
    dirs[2 * N - 1, 3] &= np.uint32((1 << 30) - 1)
    st = hm.lib().heston_price_greeks_ex(ctx.handle, ctypes.byref(cp), 0, 512, N, 1,
                                         ctypes.byref(o.c), ctypes.byref(res))
    assert st == 0


def _sobol_estimates(hm, ctx, dirs, N, n, seed, R=4):
    """heston_price_greeks_ex with the Sobol + bridge generator on the given
    direction-number table (FP64 Asian put, fused bumps)."""
    import ctypes
    o = hm._OptsHolder(hm.Options(rng=hm.SOBOL_BRIDGE, qmc_replicates=R), N)
    o.dirs = dirs
    o.c.sobol_directions = dirs.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32))
    o.c.sobol_dims = dirs.shape[0]
    res = hm.CResult()
    cp = hm._cparams(PB.__dict__)
    hm.check(hm.lib().heston_price_greeks_ex(ctx.handle, ctypes.byref(cp), hm.ASIAN_PUT, n, N,
                                             seed, ctypes.byref(o.c), ctypes.byref(res)))
    r = hm._result_dict(res)
    return {k: r[k] for k in hm.EST_NAMES}


def test_sobol_tables_kept_between_calls(hm, ctx):
    """A context keeps the seed-independent quasi-random tables from one call to
    the next.  A sequence of calls on one context that changes the step count,
    the points per replicate (64-point aligned or not, a larger per-block
    table), the direction numbers (another table, or the same array changed in
    place) and the seed gives, call by call, bitwise the results of a fresh
    context."""
    base12 = hm.sobol_directions(24)
    base20 = hm.sobol_directions(40)
    other12 = base12.copy()
    other12[1:, :30] ^= np.uint32(0x15555555) >> np.arange(30, dtype=np.uint32)
    inplace = base12.copy()
    seq = [(base12, 12, 2048, 1), (base20, 20, 2048, 2), (base12, 12, 2048, 3),
           (base12, 12, 2000, 4), (other12, 12, 2048, 5), (base12, 12, 8192, 6),
           (base12, 12, 2048, 1), (inplace, 12, 2048, 7), ("mutate", 12, 2048, 7)]
    for dirs, N, n, seed in seq:
        if isinstance(dirs, str):  # same array, new contents
            inplace[3:, 2:30] ^= np.uint32(0x2AAAAAAA) >> np.arange(2, 30, dtype=np.uint32)
            dirs = inplace
        got = _sobol_estimates(hm, ctx, dirs, N, n, seed)
        fresh = hm.Context(0)
        try:
            want = _sobol_estimates(hm, fresh, dirs, N, n, seed)
        finally:
            fresh.close()
        assert got == want, (N, n, seed)
