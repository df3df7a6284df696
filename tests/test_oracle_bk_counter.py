"""Pins of the oracle's exact (Broadie-Kaya) sampler on counter-based inputs,
the form the device sampler is checked against.

Facts outside the oracle: the gamma sampler against scipy's gamma law (KS,
shapes below and above one); the Poisson inversion against scipy's Poisson
quantile function; the variance transition against scipy's non-central
chi-square law for d > 1 and d <= 1; the European price against the
characteristic-function price (exact simulation: no discretisation bias);
the per-path put-call identity; the pathwise estimators against finite
differences of re-simulated paths.
"""
import math

import numpy as np
import pytest
from scipy import stats

import oracle
from oracle import analytic, bk
from workloads import BASE, PAPER

PB = oracle.Params(**BASE)
PP = oracle.Params(**PAPER)


@pytest.mark.parametrize("alpha", [0.134, 1.3, 5.7])
def test_gamma_sampler_law(alpha):
    g = np.array([bk.gamma_counter(alpha, 7, i, 3) for i in range(8000)])
    assert np.isfinite(g).all() and (g > 0).all()
    assert stats.kstest(g, stats.gamma(alpha).cdf).pvalue > 1e-3


def test_poisson_inversion_is_the_quantile():
    rng = np.random.default_rng(2)
    for mu in (0.01, 0.7, 3.0, 25.0, 300.0):
        for u in rng.uniform(size=200):
            assert bk.poisson_inverse(mu, u) == stats.poisson.ppf(u, mu), (mu, u)
    assert math.isnan(bk.poisson_inverse(bk.MAX_POISSON_MEAN * 1.01, 0.5))


@pytest.mark.parametrize("p", [PP, PP.replace(theta=0.004, sigma=0.7)], ids=["d>1", "d<=1"])
def test_variance_transition_law(p):
    dt, vu, n = 0.25, 0.02, 8000
    x = np.array([bk.sample_vt_counter(p, vu, dt, 11, i, 2)[0] for i in range(n)])
    e = math.exp(-p.kappa * dt)
    c = p.sigma ** 2 * (1 - e) / (4 * p.kappa)
    d = 4 * p.kappa * p.theta / p.sigma ** 2
    assert (d > 1) == (p is PP)
    assert stats.kstest(x / c, stats.ncx2(d, vu * e / c).cdf).pvalue > 1e-3


def test_draw_layout():
    """Definition check (parity unpinned: the layout is this implementation's)."""
    seed, path, step = (3 << 40) | 9, (5 << 32) | 77, 2
    w = oracle.philox(np.array([[step, 77, 5, 5 + (1 << 8)]], dtype=np.uint32),
                      np.array([[9, 3 << 8]], dtype=np.uint32))[0]
    assert np.array_equal(w, bk.draw_block(seed, path, step, 1))


def test_out_of_the_money_put_price():
    """K = 80: the skew from rho = -0.7 makes the put worth 1.14 (0.26 at rho = +0.7)."""
    q = PB.replace(K=80.0)
    n = 20_000
    rec = bk.simulate_counter(q, oracle.EURO_PUT, 1, 43, 0, n)
    m, se = oracle.mean_se(rec[:, 3])
    ref = analytic.heston_call(q) - q.S0 + q.K * math.exp(-q.r * q.T)
    assert abs(m - ref) < 4 * se


def test_orthogonal_noise_is_independent_of_the_variance():
    """rho = 0: given the variance path, ln(S_T/S0) is normal with mean r T - I/2
    and variance I (I the integral of V), independent of V_T."""
    q = PB.replace(rho=0.0)
    n = 4000
    rec, I = bk.simulate_counter(q, oracle.EURO_CALL, 1, 44, 0, n, integral=True)
    R = (np.log(rec[:, 0] / q.S0) - q.r * q.T + 0.5 * I) / np.sqrt(I)
    assert stats.kstest(R, stats.norm.cdf).pvalue > 1e-3
    assert abs(np.corrcoef(R, rec[:, 1])[0, 1]) < 4 / math.sqrt(n)


def test_european_price_is_unbiased():
    n = 20_000
    rec = bk.simulate_counter(PB, oracle.EURO_CALL, 1, 42, 0, n)
    m, se = oracle.mean_se(rec[:, 3])
    assert abs(m - analytic.heston_call(PB)) < 4 * se
    m, se = oracle.mean_se(math.exp(-PB.r * PB.T) * rec[:, 0])
    assert abs(m - PB.S0) < 4 * se


def test_put_call_identity_and_pathwise_estimators():
    n, N = 300, 4
    c = bk.simulate_counter(PP, oracle.ASIAN_CALL, N, 5, 0, n)
    q = bk.simulate_counter(PP, oracle.ASIAN_PUT, N, 5, 0, n)
    D = math.exp(-PP.r * PP.T)
    np.testing.assert_allclose(c[:, 3] - q[:, 3], D * (c[:, 2] - PP.K), rtol=0, atol=1e-12)
    h = 1e-6
    for k, name in ((4, "S0"), (5, "r")):
        x = getattr(PP, name)
        up = bk.simulate_counter(PP.replace(**{name: x + h}), oracle.ASIAN_CALL, N, 5, 0, n)[:, 3]
        dn = bk.simulate_counter(PP.replace(**{name: x - h}), oracle.ASIAN_CALL, N, 5, 0, n)[:, 3]
        away = np.abs(c[:, 2] - PP.K) > 1e-3 * PP.K
        np.testing.assert_allclose(c[away, k], ((up - dn) / (2 * h))[away], rtol=1e-5, atol=1e-7)
