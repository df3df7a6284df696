"""Pins of the oracle's quadratic-exponential (QE) path (no GPU needed).

The paper names Andersen's QE scheme as future work for the variance
process; the oracle follows Andersen (2008).  Each test checks it against a
fact outside the oracle: the exact transition law of the square-root process
(scipy's non-central chi-square), the binomial law of the point mass at zero,
the characteristic-function price of the Heston model, the martingale
property of the discounted price, and the per-path put-call identity.
"""
import math

import numpy as np
import pytest
from scipy import stats

import oracle
from oracle import analytic
from workloads import BASE

PB = oracle.Params(**BASE)
EC, EP, AC, AP = oracle.EURO_CALL, oracle.EURO_PUT, oracle.ASIAN_CALL, oracle.ASIAN_PUT


def cir_transition(p, V, dt):
    """Exact law of V(t+dt) given V(t) = V: c times a non-central chi-square
    with d = 4 kappa theta / sigma^2 degrees of freedom and non-centrality
    V e^{-kappa dt} / c, c = sigma^2 (1 - e^{-kappa dt}) / (4 kappa)."""
    c = p.sigma ** 2 * (1.0 - math.exp(-p.kappa * dt)) / (4.0 * p.kappa)
    d = 4.0 * p.kappa * p.theta / p.sigma ** 2
    lam = V * math.exp(-p.kappa * dt) / c
    return stats.ncx2(d, lam, scale=c)


def one_step(p, n, seed=3):
    """V after one QE step of length T from v0, for n paths."""
    rec, _, _ = oracle.simulate_qe(p, EC, 1, seed, 0, n, threads=8)
    return rec[:, 1]


@pytest.mark.parametrize("case", ["quadratic", "exponential"])
def test_one_step_matches_cir_mean_and_variance(case):
    """QE matches the first two conditional moments of the exact transition:
    the sample mean and variance of one step agree with scipy's non-central
    chi-square moments.  psi = s^2 / m^2 is below 3/2 in the first case (scaled
    squared normal) and above it in the second (point mass at 0 + exponential)."""
    if case == "quadratic":
        p = PB.replace(T=0.25, v0=0.04, sigma=0.3)
    else:
        p = PB.replace(T=1.0, v0=0.01, kappa=0.5, theta=0.02, sigma=1.0)
    law = cir_transition(p, p.v0, p.T)
    m, s2 = law.mean(), law.var()
    psi = s2 / m ** 2
    assert (psi <= 1.5) == (case == "quadratic")
    n = 400_000
    v = one_step(p, n)
    assert (v >= 0).all()
    se_mean = math.sqrt(s2 / n)
    assert abs(v.mean() - m) < 4.5 * se_mean
    # standard error of the sample variance from the sample's fourth moment
    mu4 = ((v - v.mean()) ** 4).mean()
    se_var = math.sqrt(max(mu4 - v.var() ** 2, 0.0) / n)
    assert abs(v.var() - s2) < 4.5 * se_var


def test_exponential_branch_mass_at_zero():
    """In the exponential branch V(t+dt) = 0 with probability p = (psi-1)/(psi+1),
    psi from the exact conditional moments: the fraction of zeros is binomial."""
    p = PB.replace(T=1.0, v0=0.01, kappa=0.5, theta=0.02, sigma=1.0)
    law = cir_transition(p, p.v0, p.T)
    psi = law.var() / law.mean() ** 2
    pz = (psi - 1.0) / (psi + 1.0)
    n = 400_000
    v = one_step(p, n, seed=9)
    frac = (v == 0.0).mean()
    assert abs(frac - pz) < 4.5 * math.sqrt(pz * (1 - pz) / n)


def test_draw_layout():
    """Definition check (parity unpinned: the layout is this implementation's):
    step j of path k takes the Philox block with counter (j, lo32 k, hi32 k, 4);
    words 0, 1 give the Box-Muller pair (Zs, Zv) and word 2 the uniform Uv."""
    seed, path, step = (5 << 40) | 17, (3 << 32) | 123, 77
    w = oracle.philox(np.array([[step, path & 0xFFFFFFFF, path >> 32, 4]], dtype=np.uint32),
                      np.array([[seed & 0xFFFFFFFF, seed >> 32]], dtype=np.uint32))[0]
    u = [((int(x) >> 9) + 0.5) * 2.0 ** -23 for x in w]
    r = math.sqrt(-2.0 * math.log(u[0]))
    zs, zv, uv = oracle.qe_draws(seed, path, step)
    assert zs == pytest.approx(r * math.cos(2 * math.pi * u[1]), abs=1e-14)
    assert zv == pytest.approx(r * math.sin(2 * math.pi * u[1]), abs=1e-14)
    assert uv == u[2]


@pytest.mark.parametrize("p", [PB, PB.replace(kappa=0.5, theta=0.02, sigma=1.0, v0=0.02)])
def test_qe_european_matches_analytic(p):
    """The QE price converges with few steps: 32 steps are within 3.5 standard
    errors plus the step-halving difference of the characteristic-function price,
    also where the Feller condition fails badly (second case)."""
    n = 400_000
    ref = analytic.heston_call(p)
    r32, _, _ = oracle.simulate_qe(p, EC, 32, 11, 0, n, threads=8)
    r16, _, _ = oracle.simulate_qe(p, EC, 16, 11, 0, n, threads=8)
    m32, se32 = oracle.mean_se(r32[:, 3])
    m16, _ = oracle.mean_se(r16[:, 3])
    assert abs(m32 - ref) < 3.5 * se32 + abs(m32 - m16)


def test_qe_martingale():
    """e^{-rT} E[S_T] = S0 within the statistical error (the scheme without the
    martingale correction leaves a bias far below it at these parameters)."""
    n = 400_000
    rec, _, _ = oracle.simulate_qe(PB, EC, 24, 5, 0, n, threads=8)
    disc = math.exp(-PB.r * PB.T) * rec[:, 0]
    m, se = oracle.mean_se(disc)
    assert abs(m - PB.S0) < 4.0 * se


@pytest.mark.parametrize("asian", [False, True])
def test_qe_put_call_identity_per_path(asian):
    """Same paths for the call and the put: C - P = D (X - K) on every path."""
    c, _, _ = oracle.simulate_qe(PB, AC if asian else EC, 12, 4, 0, 2000)
    q, _, _ = oracle.simulate_qe(PB, AP if asian else EP, 12, 4, 0, 2000)
    D = math.exp(-PB.r * PB.T)
    np.testing.assert_allclose(c[:, 3] - q[:, 3], D * (c[:, 2] - PB.K), rtol=0, atol=1e-12)
    np.testing.assert_array_equal(c[:, 0], q[:, 0])


def test_qe_rejects_unsupported_inputs():
    with pytest.raises(ValueError):
        oracle.simulate_qe(PB.replace(sigma=0.0), EC, 4, 1, 0, 10)
    with pytest.raises(ValueError):
        oracle.simulate_qe(PB.replace(theta=0.0), EC, 4, 1, 0, 10)


def test_amplification_bounds_a_whole_path_difference():
    """amp bounds, in units of the variance scale max(V_T, v0, theta), the growth of
    a relative perturbation of v0 into V_T, which a central difference of whole
    re-simulated paths in v0 measures directly."""
    p = PB.replace(kappa=0.5, theta=0.02, sigma=1.0, v0=0.02)
    n, N, h = 400, 12, 1e-6
    rec, margin, amp = oracle.simulate_qe(p, EC, N, 21, 0, n)
    up, _, _ = oracle.simulate_qe(p.replace(v0=p.v0 * (1 + h)), EC, N, 21, 0, n)
    dn, _, _ = oracle.simulate_qe(p.replace(v0=p.v0 * (1 - h)), EC, N, 21, 0, n)
    growth = np.abs(up[:, 1] - dn[:, 1]) / (2 * h) / np.maximum(rec[:, 1], max(p.v0, p.theta))
    ok = margin > 1e-3
    assert ok.mean() > 0.5
    assert (amp[ok] >= 0.999 * growth[ok] - 1e-9).all()
    assert (amp >= 1.0).all() and amp.max() > 5.0
