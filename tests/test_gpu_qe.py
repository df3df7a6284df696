"""GPU parity of the quadratic-exponential (QE) scheme against the oracle.

Per path (heston_dump_paths records written by the pricing kernel) against
oracle.simulate_qe on the same Philox inputs, with the per-path bar of the
Milstein parity tests (tol max(|oracle|, floor), tol 1e-12 in FP64 and 1e-5
in FP32).  QE chooses a branch per step by comparing psi = s^2/m^2 with 3/2
and, in the exponential branch, the uniform with the mass p at zero; each
side takes those decisions in its own precision, so a path may only differ
where the oracle's decision margin (the smallest such distance along the
path) is below 1e-9 (FP64) or 1e-4 (FP32); such paths must stay rare.

The FP64 bar is the plain 1e-12.  In binary32 a QE path can sit further
than 1e-5 from the FP64 oracle for reasons of arithmetic alone: a QE variance
step from a small variance into a large one amplifies earlier relative errors
of the variance (|dV'/dV| above 10 where vol of vol is high), and every later
log-price increment uses those variances.  tests/qe_binary32.py evaluates the
kernel's formulas in binary32 on the CPU, and tests/test_qe_binary32.py shows
there that such evaluations miss 1e-5 on amplified paths, by amounts that grow
with the oracle's amplification a_p, and that three times the spread of a
16-member Monte-Carlo-arithmetic ensemble bounds other binary32 evaluations.
The FP32 bar per path and column is therefore
max(1e-5 max(|oracle|, floor), 3 x that spread): where binary32 itself is
exact to 1e-5 it is the plain bar, and nowhere is it wider than what a
binary32 evaluation on the CPU shows for the same path.
"""
import math

import numpy as np
import pytest

import oracle
import qe_binary32
from oracle import analytic
from workloads import BASE

pytestmark = pytest.mark.gpu

PB = oracle.Params(**BASE)
# vol of vol well above the Feller bound: the exponential branch is frequent
PF = PB.replace(kappa=0.5, theta=0.02, sigma=1.0, v0=0.02)
TOL = {0: 1e-12, 1: 1e-5}
MARGIN = {0: 1e-9, 1: 1e-4}


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


def compare(name, g, o, bar, skip):
    err = np.abs(g - o)
    bad = (err > bar) & ~skip
    if bad.any():
        i = int(np.argmax(np.where(bad, err / bar, 0)))
        raise AssertionError(f"{name}: {int(bad.sum())} paths off, worst path {i}: "
                             f"gpu {g[i]!r} oracle {o[i]!r} |d| {err[i]:.3e} > bar {bar[i]:.3e}")


def check(hm, ctx, p, opt_type, n, N, seed, prec, first=0, bumps=True, n_total=None):
    """Dumped records of paths first .. first+n-1 (of a launch over n_total
    paths, default first + n) against the oracle's, every column (bump
    scenarios re-simulated by the oracle)."""
    tol = TOL[prec]
    opts = hm.Options(precision=prec, scheme=hm.QE,
                      greeks=hm.GREEKS_PATHWISE | (hm.GREEKS_BUMP_FUSED if bumps else 0))
    d = ctx.dump_paths(p.__dict__, opt_type, n_total or first + n, N, seed, first, n,
                       opts).cpu().numpy()
    rec, margin, _ = oracle.simulate_qe(p, opt_type, N, seed, first, n, threads=8)
    k = 14 if bumps else 6
    ref = np.empty((n, k))
    ref[:, :6] = rec
    skip = margin < MARGIN[prec]
    base_skip = skip.copy()
    if bumps:
        for i, (_, q) in enumerate(list(oracle.scenario_params(p, oracle.Bumps()).items())[1:]):
            r, m, _ = oracle.simulate_qe(q, opt_type, N, seed, first, n, threads=8)
            ref[:, 6 + i] = r[:, 3]
            skip |= m < MARGIN[prec]
    else:
        assert np.isnan(d[:, 6:14]).all()
    vfloor = max(p.v0, p.theta)
    floors = np.array([p.S0, vfloor, p.S0, p.S0, 1.0, p.K * p.T] + [p.S0] * 8)[:k]
    bar = tol * np.maximum(np.abs(ref), floors)
    if prec == 1:
        bar = np.maximum(bar, 3 * qe_binary32.spread(p, opt_type, N, seed, first, n, ref, bumps,
                                                      members=16))
    near = np.abs(ref[:, 2] - p.K) < 1e3 * tol * p.K
    names = list(oracle.REC_FIELDS) + ["pay_" + sc for sc in oracle.SCENARIOS[1:]]
    for c in range(k):
        sk = (base_skip if c < 6 else skip) | (near if names[c] in ("pw_delta", "pw_rho") else False)
        compare(names[c], d[:, c], ref[:, c], bar[:, c], sk)
    assert skip.mean() < 0.01, f"{skip.mean():.3%} of paths near a branch decision"
    return d, rec


@pytest.mark.parametrize("opt_type", [0, 1, 2, 3, 4, 5])
@pytest.mark.parametrize("p", [PB, PF], ids=["feller", "high-vol-of-vol"])
def test_qe_fp64_parity(hm, ctx, p, opt_type):
    check(hm, ctx, p, opt_type, 1037, 13, 42, 0)


@pytest.mark.parametrize("p", [PB, PF], ids=["feller", "high-vol-of-vol"])
def test_qe_fp32_parity(hm, ctx, p):
    for t in (0, 2, 4):
        check(hm, ctx, p, t, 4099, 24, 7, 1)


def test_qe_fp32_full_size_sampled_and_reduction(hm, ctx):
    """The 2^20-path x 252-step FP32 Asian call under QE with five bump Greeks,
    in the launch the benchmark times: sampled windows against the oracle
    (every column, the same bar as above), and the reduced estimates against
    the host sums of every path's dumped record."""
    n, N, seed = 1 << 20, 252, 42
    opts = hm.Options(precision=hm.FP32, scheme=hm.QE)
    r = ctx.price_greeks(PB.__dict__, hm.ASIAN_CALL, n, N, seed, opts)
    full = ctx.dump_paths(PB.__dict__, hm.ASIAN_CALL, n, N, seed, 0, n, opts).cpu().numpy()
    for first in (0, n // 2 + 12345, n - 512):
        d, _ = check(hm, ctx, PB, hm.ASIAN_CALL, 512, N, seed, 1, first=first, n_total=n)
        np.testing.assert_array_equal(d, full[first:first + 512])
    pay = {sc: full[:, 6 + k] for k, sc in enumerate(oracle.SCENARIOS[1:])}
    pay["base"] = full[:, 3]
    samples = oracle.greek_samples(pay, PB)
    samples["pw_delta"], samples["pw_rho"] = full[:, 4], full[:, 5]
    for k, y in samples.items():
        m, se = oracle.mean_se(y)
        assert r[k][0] == pytest.approx(m, rel=1e-9, abs=1e-12), k
        assert r[k][1] == pytest.approx(se, rel=1e-6), k


def test_qe_exponential_branch_is_exercised(hm, ctx):
    """The high vol-of-vol case ends many paths at exactly zero variance, on both sides."""
    d, rec = check(hm, ctx, PF, 0, 2048, 8, 3, 0, bumps=False)
    zeros = rec[:, 1] == 0.0
    assert zeros.mean() > 0.2
    assert (d[zeros, 1] == 0.0).mean() > 0.99


def test_qe_path_above_2_32(hm, ctx):
    check(hm, ctx, PB, 2, 300, 7, (7 << 40) | 3, 0, first=(1 << 32) + 5, bumps=False)


def test_qe_estimates_match_oracle_and_analytic(hm, ctx):
    """Reduced estimates equal the host sums of the oracle's per-path values, and
    the FP32 price on 2^20 paths x 32 steps sits within 3.5 standard errors (plus
    the step-halving difference) of the characteristic-function price."""
    n, N = 20_000, 16
    opts = hm.Options(precision=hm.FP64, scheme=hm.QE, greeks=hm.GREEKS_PATHWISE)
    r = ctx.price_greeks(PB.__dict__, 0, n, N, 5, opts)
    rec, _, _ = oracle.simulate_qe(PB, 0, N, 5, 0, n, threads=8)
    m, se = oracle.mean_se(rec[:, 3])
    assert r["price"][0] == pytest.approx(m, rel=1e-10)
    assert r["price"][1] == pytest.approx(se, rel=1e-6)
    big = hm.Options(precision=hm.FP32, scheme=hm.QE, greeks=hm.GREEKS_PATHWISE)
    r32 = ctx.price_greeks(PB.__dict__, 0, 1 << 20, 32, 9, big)
    r16 = ctx.price_greeks(PB.__dict__, 0, 1 << 20, 16, 9, big)
    ref = analytic.heston_call(PB)
    assert abs(r32["price"][0] - ref) < 3.5 * r32["price"][1] + abs(r32["price"][0] - r16["price"][0])


def test_qe_rejections(hm, ctx):
    qe = hm.Options(scheme=hm.QE)
    with pytest.raises(hm.HestonError) as e:
        ctx.price_greeks(PB.replace(sigma=0.0).__dict__, 0, 100, 4, 1, qe)
    assert e.value.status == -1
    with pytest.raises(hm.HestonError) as e:
        ctx.price_greeks(PB.__dict__, 0, 64, 4, 1,
                         hm.Options(scheme=hm.QE, rng=hm.SOBOL_BRIDGE, qmc_replicates=2))
    assert e.value.status == -5
    # batches take QE (tests/test_gpu_batch.py), with the same parameter checks
    with pytest.raises(hm.HestonError) as e:
        ctx.price_batch([dict(params=PB.replace(sigma=0.0).__dict__, type=0, n_steps=4,
                              n_paths=100, seed=1, want=1)], qe)
    assert e.value.status == -1
