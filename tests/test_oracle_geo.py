"""Pins of the geometric-average Asian options (the paper notes that the
average may be arithmetic or geometric) and of their semi-analytic price.

Facts outside the oracle: the arithmetic-geometric mean inequality on every
path; the per-path put-call identity; pathwise Delta and Rho as exact
derivatives (central differences of re-simulated paths); for the transform
price, its reduction to the European characteristic-function price for one
fixing date and to a Black-Scholes form with deterministic variance as the vol
of vol vanishes; and the Monte-Carlo price of the oracle's Milstein paths.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import analytic
from workloads import BASE

PB = oracle.Params(**BASE)
GC, GP, AC = oracle.GEO_ASIAN_CALL, oracle.GEO_ASIAN_PUT, oracle.ASIAN_CALL


def test_transform_price_with_one_fixing_is_the_european_price():
    for p in (PB, PB.replace(rho=0.3, sigma=0.6, v0=0.02)):
        assert analytic.geometric_asian_call(p, [p.T]) == pytest.approx(analytic.heston_call(p),
                                                                        rel=1e-10)


def test_transform_price_deterministic_variance_limit():
    """sigma -> 0: a Richardson step over sigma = 2e-4, 1e-4 reaches the normal
    log-average (Black-Scholes) form with V_t = theta + (v0 - theta) e^{-kappa t}."""
    p = PB.replace(v0=0.02, theta=0.05)
    t = np.arange(1, 13) / 12
    ref = analytic.geometric_asian_call_deterministic_variance(p.replace(sigma=0.0), t)
    a = analytic.geometric_asian_call(p.replace(sigma=2e-4), t)
    b = analytic.geometric_asian_call(p.replace(sigma=1e-4), t)
    assert 2 * b - a == pytest.approx(ref, rel=1e-6)


def test_geometric_not_above_arithmetic_on_every_path():
    g = oracle.simulate(PB, GC, 24, 3, 0, 2000)
    a = oracle.simulate(PB, AC, 24, 3, 0, 2000)
    np.testing.assert_array_equal(g[:, 0], a[:, 0])  # same paths
    assert (g[:, 2] <= a[:, 2] * (1 + 1e-15)).all()
    assert (g[:, 2] < a[:, 2]).mean() > 0.99


def test_geometric_put_call_identity_per_path():
    c = oracle.simulate(PB, GC, 24, 4, 0, 2000)
    q = oracle.simulate(PB, GP, 24, 4, 0, 2000)
    D = math.exp(-PB.r * PB.T)
    np.testing.assert_allclose(c[:, 3] - q[:, 3], D * (c[:, 2] - PB.K), rtol=0, atol=1e-12)


@pytest.mark.parametrize("opt", [GC, GP])
def test_geometric_pathwise_estimators_are_exact_derivatives(opt):
    n, N, seed = 400, 12, 8
    rec = oracle.simulate(PB, opt, N, seed, 0, n)
    h = 1e-6
    for k, name in ((4, "S0"), (5, "r")):
        x = getattr(PB, name)
        up = oracle.simulate(PB.replace(**{name: x + h}), opt, N, seed, 0, n)[:, 3]
        dn = oracle.simulate(PB.replace(**{name: x - h}), opt, N, seed, 0, n)[:, 3]
        fd = (up - dn) / (2 * h)
        away = np.abs(rec[:, 2] - PB.K) > 1e-3 * PB.K  # no kink between the bumps
        np.testing.assert_allclose(rec[away, k], fd[away], rtol=1e-6, atol=1e-8)


@pytest.mark.parametrize("fix", ["monthly", "daily"])
def test_geometric_monte_carlo_matches_transform_price(fix):
    N = 252
    steps = np.arange(21, 253, 21) if fix == "monthly" else np.arange(1, 253)
    t = steps / N * PB.T
    ref = analytic.geometric_asian_call(PB, t)
    n = 100_000
    r = oracle.simulate(PB, GC, N, 13, 0, n, fixings=steps, threads=8)
    m, se = oracle.mean_se(r[:, 3])
    # the same dates on a grid twice as fine bounds the discretisation bias
    h = oracle.simulate(PB, GC, 2 * N, 13, 0, n, fixings=2 * steps, threads=8)
    mh, _ = oracle.mean_se(h[:, 3])
    assert abs(m - ref) < 3.5 * se + abs(m - mh)


def test_geometric_tangent_rejected():
    with pytest.raises(ValueError):
        oracle.tangent(PB, GC, 4, 1, 0, 10)
