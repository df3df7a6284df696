"""Why the adjoint parity bars are max(tol max(|o|, floor), 4 x spread).

The GPU adjoint tests compare each path's payoff and its seven derivatives
with the oracle's forward-mode derivatives (tol 1e-12 in FP64, 1e-5 in FP32;
floors as ``tangent_binary32.floors``).  Where the variance comes close to zero
the Milstein variance map amplifies relative rounding errors, so no
evaluation in the working precision can meet the plain bar on such paths.
``tests/tangent_binary32.py`` evaluates the same derivatives in binary32 or
binary64 with Monte Carlo arithmetic; its ``spread`` (largest distance from
the oracle over the round-to-nearest and sixteen randomly rounded evaluations)
is the per-path allowance.  These CPU tests show what the bar rests on:

- the evaluation is the oracle's arithmetic (binary64, well-conditioned
  parameters: equal to 1e-13);
- with the Feller condition satisfied the plain FP32 bar holds on every path,
  and the bar stays within 1.5 times the plain one;
- at vol of vol 0.6 (Feller violated) a round-to-nearest binary32 evaluation
  misses the plain bar, on paths whose variance came close to zero;
- four times the sixteen-member spread covers further, independently rounded
  evaluations in both precisions, and a differently ordered binary64 one.
"""
import numpy as np
import pytest

import oracle
import workloads
from workloads import BASE

import tangent_binary32 as tb

PB = oracle.Params(**BASE)
PV = PB.replace(sigma=0.6)  # 2 kappa theta / sigma^2 = 0.44


def near_strike(p, t, N, seed, n, mode=oracle.FULL_TRUNC, fix=None, tol=1e-5):
    rec = oracle.simulate(p, t, N, seed, 0, n, mode, fix, threads=8)
    return np.abs(rec[:, 2] - p.K) < 1e3 * tol * p.K


@pytest.mark.parametrize("t", [0, 1, 2, 3])
@pytest.mark.parametrize("mode", [oracle.FULL_TRUNC, oracle.ABSORB])
def test_fp64_evaluation_reproduces_oracle(t, mode):
    """Vol of vol 0.45: variances come within a few 1e-5 of zero (a_p near 20),
    so both truncations' branches are taken, yet every path is conditioned well
    enough for two binary64 evaluations to agree to 1e-13."""
    p = PB.replace(sigma=0.45)
    N, n = 37, 1500
    fix = (3, 10, 20, 37) if t >= 2 else None
    tan = oracle.tangent(p, t, N, 11, 0, n, mode, fix, threads=8)
    ev = tb.evaluate(p, t, N, 11, 0, n, mode, fix, dtype=np.float64)
    rel = np.abs(ev[:, :8] - tan[:, :8]) / np.maximum(np.abs(tan[:, :8]), tb.floors(p))
    assert rel.max() < 1e-13, rel.max()
    assert np.array_equal(ev[:, 8] > 0, tan[:, 8] > 0)


def test_binary32_meets_plain_bar_when_feller_holds():
    """Base parameters (2 kappa theta / sigma^2 = 1.8): the round-to-nearest
    binary32 evaluation stays inside 1e-5 max(|o|, floor) on every path away
    from the strike, and the spread stays below half that bar, so the parity
    bar is at most 1.5 times the plain one."""
    N, n = 100, 4196
    for t in (0, 2):
        tan = oracle.tangent(PB, t, N, 5, 0, n, threads=8)
        ev = tb.evaluate(PB, t, N, 5, 0, n)
        ok = ~near_strike(PB, t, N, 5, n)
        plain = 1e-5 * np.maximum(np.abs(tan[:, :8]), tb.floors(PB))
        assert (np.abs(ev[:, :8] - tan[:, :8])[ok] <= plain[ok]).all()
        s = tb.spread(PB, t, N, 5, 0, n, tan)
        assert (s[ok] <= 0.5 * plain[ok]).all()


def test_binary32_misses_plain_bar_where_variance_nears_zero():
    """Vol of vol 0.6: the round-to-nearest binary32 evaluation misses the
    plain bar on some paths, and those paths are the ones whose variance came
    close to zero (the largest sqrt(dt / V+) / 2 on the path, a_p)."""
    N, n = 100, 4196
    tan = oracle.tangent(PV, 0, N, 5, 0, n, threads=8)
    ev = tb.evaluate(PV, 0, N, 5, 0, n)
    ok = ~near_strike(PV, 0, N, 5, n)
    plain = 1e-5 * np.maximum(np.abs(tan[:, :8]), tb.floors(PV))
    miss = ((np.abs(ev[:, :8] - tan[:, :8]) > plain).any(axis=1)) & ok
    assert miss.sum() >= 10
    assert np.median(tan[miss, 8]) > 2 * np.median(tan[ok, 8])


def test_binary32_misses_plain_bar_in_serving_requests():
    """A request of the serving workload that violates the Feller condition
    (2 kappa theta / sigma^2 = 0.11), as the served FP32 adjoint runs it."""
    rs = workloads.request_stream(12, 1.0, seed=9)
    i = 11
    p = oracle.Params(**rs.params[i])
    assert 2 * p.kappa * p.theta / p.sigma ** 2 < 0.2
    t, N, seed, n = int(rs.opt_type[i]), int(rs.n_steps[i]), int(rs.seed[i]), 1024
    tan = oracle.tangent(p, t, N, seed, 0, n, threads=8)
    ev = tb.evaluate(p, t, N, seed, 0, n)
    ok = ~near_strike(p, t, N, seed, n)
    plain = 1e-5 * np.maximum(np.abs(tan[:, :8]), tb.floors(p))
    assert ((np.abs(ev[:, :8] - tan[:, :8]) > plain).any(axis=1) & ok).any()


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_bar_covers_further_evaluations(dtype):
    """Vol of vol 0.6: sixteen further Monte-Carlo-arithmetic evaluations
    (independent seeds) land within the bar (4 x the sixteen-member spread)
    of the oracle, on every path and column away from the strike."""
    N, n = 100, 4196
    for t in (0, 2):
        tan = oracle.tangent(PV, t, N, 5, 0, n, threads=8)
        bar = tb.bars(PV, t, N, 5, 0, n, tan, dtype=dtype)
        z = oracle.normals(5, 0, n, N)
        ok = ~near_strike(PV, t, N, 5, n)
        for m in range(16):
            ev = tb.evaluate(PV, t, N, 5, 0, n, dtype=dtype, mca_seed=9000 + m,
                             normals=z)
            worst = (np.abs(ev[:, :8] - tan[:, :8]) / bar)[ok].max()
            assert worst <= 1.0, (t, m, worst)


def test_fp64_spread_covers_the_oracles_own_rounding():
    """FP64, vol of vol 0.6 at the GPU parity test's size: the oracle and the
    binary64 evaluation round in different orders and differ by more than
    1e-12 relative on some paths; 4 x the binary64 spread covers it."""
    N, n = 37, 2013
    tan = oracle.tangent(PV, 0, N, 11, 0, n, threads=8)
    ev = tb.evaluate(PV, 0, N, 11, 0, n, dtype=np.float64)
    d = np.abs(ev[:, :8] - tan[:, :8])
    plain = 1e-12 * np.maximum(np.abs(tan[:, :8]), tb.floors(PV))
    assert (d > plain).any()
    # the round-to-nearest evaluation is part of the spread, so compare with
    # the randomly rounded members alone
    z = oracle.normals(11, 0, n, N)
    s = np.zeros_like(d)
    for m in range(tb.MEMBERS):
        v = tb.evaluate(PV, 0, N, 11, 0, n, dtype=np.float64, mca_seed=1 + m,
                        normals=z)
        s = np.fmax(s, np.abs(v[:, :8] - tan[:, :8]))
    assert (d <= np.maximum(plain, tb.FACTOR * s)).all()


# ---------------------------------------------------------------------------
# Andersen's QE scheme: the same bars for the QE adjoint.

PQ = PB.replace(sigma=0.9, kappa=1.0, theta=0.05)  # Feller violated: exponential branch, zero mass


@pytest.mark.parametrize("t", [0, 1, 2, 3])
def test_qe_fp64_evaluation_reproduces_oracle(t):
    """The QE evaluation is the oracle's QE tangent in binary64 (base
    parameters, explicit fixings for the Asians)."""
    N, n = 37, 1500
    fix = (3, 10, 20, 37) if t >= 2 else None
    tan = oracle.tangent(PB, t, N, 11, 0, n, oracle.QE, fix, threads=8)
    ev = tb.evaluate(PB, t, N, 11, 0, n, oracle.QE, fix, dtype=np.float64)
    rel = np.abs(ev[:, :8] - tan[:, :8]) / np.maximum(np.abs(tan[:, :8]), tb.floors(PB))
    assert rel.max() < 1e-13, rel.max()


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_qe_bar_covers_further_evaluations(dtype):
    """Feller violated: sixteen further Monte-Carlo-arithmetic QE evaluations
    land within the bar on every path and column away from the strike and from
    a branch switch (margin 1e-4 in binary32, 1e-9 in binary64)."""
    N, n = 100, 4196
    for t in (0, 2):
        tan = oracle.tangent(PQ, t, N, 5, 0, n, oracle.QE, threads=8)
        bar = tb.bars(PQ, t, N, 5, 0, n, tan, oracle.QE, dtype=dtype)
        z = tb.inputs(PQ, t, N, 5, 0, n, oracle.QE)
        single = dtype == np.float32
        ok = ~near_strike(PQ, t, N, 5, n, oracle.QE, tol=1e-5 if single else 1e-12)
        ok &= tan[:, 8] >= (1e-4 if single else 1e-9)
        assert ok.mean() > 0.9
        for m in range(16):
            ev = tb.evaluate(PQ, t, N, 5, 0, n, oracle.QE, dtype=dtype, mca_seed=9000 + m,
                             normals=z)
            worst = (np.abs(ev[:, :8] - tan[:, :8]) / bar)[ok].max()
            assert worst <= 1.0, (t, m, worst)
