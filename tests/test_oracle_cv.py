"""Pins of the oracle's geometric-average control variate for the arithmetic
Asian price (Kemna and Vorst, 1990; the paper notes the average may be
geometric).

Facts outside the oracle: with one fixing date the two averages coincide, so
the estimator must return the characteristic-function European price exactly
with zero error; beta and the standard error are those of the least-squares
line of the arithmetic payoff on the geometric one (numpy's polyfit); the
paper's exact-simulation value of the quarterly Asian; equal-size replicates
give the same estimate as the pooled paths (linearity).
"""
import math

import numpy as np
import pytest

import oracle
from oracle import analytic
from workloads import BASE, PAPER, paper_fixing_steps

PB = oracle.Params(**BASE)
PP = oracle.Params(**PAPER)
AC, AP = oracle.ASIAN_CALL, oracle.ASIAN_PUT


@pytest.mark.parametrize("opt", [AC, AP])
def test_one_fixing_returns_the_european_price_exactly(opt):
    N = 16
    est, se, beta, mu, a, g = oracle.cv_price(PB, opt, 4000, N, 5, fixings=(N,), threads=8)
    np.testing.assert_allclose(a, g, rtol=1e-13, atol=1e-13)
    ref = analytic.heston_call(PB)
    if opt == AP:
        ref -= PB.S0 - PB.K * math.exp(-PB.r * PB.T)
    assert beta == pytest.approx(1.0, abs=1e-10)
    assert est == pytest.approx(ref, rel=1e-9)
    assert se < 1e-10 * PB.S0


@pytest.mark.parametrize("opt", [AC, AP])
def test_beta_and_error_are_the_least_squares_line(opt):
    n = 20_000
    est, se, beta, mu, a, g = oracle.cv_price(PB, opt, n, 24, 3, threads=8)
    slope, icpt = np.polyfit(g, a, 1)
    assert beta == pytest.approx(slope, rel=1e-10)
    resid = a - (slope * g + icpt)
    assert se == pytest.approx(math.sqrt((resid ** 2).sum() / (n - 1) / n), rel=1e-8)
    # the line through (mu, icpt + slope mu) is the estimate
    assert est == pytest.approx(icpt + slope * mu, rel=1e-10)
    _, se_plain = oracle.mean_se(a)
    assert se < 0.2 * se_plain


def test_matches_paper_exact_simulation_quarterly_asian():
    """Paper parameters, quarterly fixings, absorption, 128 steps: the paper's
    exact-simulation value 4.3840 (0.0064)."""
    N = 128
    est, se, *_ = oracle.cv_price(PP, AC, 1 << 16, N, 29, mode=oracle.ABSORB,
                                  fixings=paper_fixing_steps(N), threads=8)
    assert abs(est - 4.3840) < 3 * math.hypot(se, 0.0064)


def test_replicates_give_the_pooled_estimate():
    rng = np.random.default_rng(1)
    g = rng.lognormal(size=4096)
    a = 1.1 * g + 0.1 * rng.normal(size=4096)
    e1, _, b1 = oracle.control_variate(a, g, 1.7)
    e2, se2, b2 = oracle.control_variate_reps(a, g, 1.7, 8)
    assert e2 == pytest.approx(e1, rel=1e-13)
    assert b2 == b1
    r = (a.reshape(8, -1).mean(1) - b1 * (g.reshape(8, -1).mean(1) - 1.7))
    assert se2 == pytest.approx(r.std(ddof=1) / math.sqrt(8), rel=1e-12)


def test_control_mean_needs_an_arithmetic_asian():
    with pytest.raises(ValueError):
        oracle.geometric_control_mean(PB, oracle.EURO_CALL, 4)
