"""Pins of the oracle's partial-truncation and reflection modes (Lord, Koekkoek
and van Dijk 2010; the paper itself uses absorption).  Facts outside the
oracle: the second variance step differs from full truncation's by an amount
fixed by the first step's variance and the pinned Philox normals; all fixes
coincide with full truncation where the variance never turns negative; each
converges to the characteristic-function price; the martingale property.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import analytic
from workloads import BASE

PB = oracle.Params(**BASE)
EC = oracle.EURO_CALL
# vol of vol high enough that the first step often turns the variance negative
PN = PB.replace(v0=0.01, sigma=1.0, kappa=1.0, theta=0.02)


def two_steps(mode, n=4000, seed=19):
    return oracle.simulate(PN, EC, 2, seed, 0, n, mode)


def test_second_step_against_full_truncation():
    """With V1 the variance after the first step (a one-step run over T/2 on the
    same normals) and dt = T/2: the log-price step of reflection adds
    -|V1| dt / 2 + sqrt(|V1| dt) Z1 where V1 < 0 (full truncation adds nothing
    there), partial truncation's equals full truncation's; partial truncation's V2 exceeds full
    truncation's by -kappa dt V1 where V1 < 0 (its drift uses V1 itself), and
    reflection's by |V1| - V1 - kappa dt |V1| + sigma sqrt(|V1| dt) Z2 (all of its
    uses take |V1|); both equal full truncation where V1 >= 0."""
    n, seed = 4000, 19
    dt = PN.T / 2
    V1 = oracle.simulate(PN.replace(T=dt), EC, 1, seed, 0, n, oracle.FULL_TRUNC)[:, 1]
    za, zb = oracle.normals(seed, 0, n, 2)
    z2 = PN.rho * za[:, 1] + math.sqrt(1 - PN.rho ** 2) * zb[:, 1]
    recs = [two_steps(m, n, seed) for m in (oracle.FULL_TRUNC, oracle.PARTIAL_TRUNC, oracle.REFLECT)]
    ft, pt, rf = (r[:, 1] for r in recs)
    neg = V1 < 0
    # the log-price step takes f3: max(V1, 0) for full and partial truncation,
    # |V1| for reflection
    z1 = za[:, 1]
    np.testing.assert_array_equal(recs[1][:, 0], recs[0][:, 0])
    dln = np.log(recs[2][:, 0] / recs[0][:, 0])
    a1 = np.abs(V1)
    np.testing.assert_allclose(dln, np.where(neg, -0.5 * a1 * dt + np.sqrt(a1 * dt) * z1, 0.0),
                               rtol=0, atol=1e-13)
    assert 0.1 < neg.mean() < 0.9
    np.testing.assert_allclose(pt - ft, np.where(neg, -PN.kappa * dt * V1, 0.0), rtol=0, atol=1e-14)
    a = np.abs(V1)
    want = np.where(neg, a - V1 - PN.kappa * dt * a + PN.sigma * np.sqrt(a * dt) * z2, 0.0)
    np.testing.assert_allclose(rf - ft, want, rtol=0, atol=1e-14)


def test_fixes_coincide_while_variance_stays_positive():
    p = PB.replace(sigma=0.05)
    ref = oracle.simulate(p, oracle.ASIAN_CALL, 16, 2, 0, 500, oracle.FULL_TRUNC)
    for m in (oracle.PARTIAL_TRUNC, oracle.REFLECT, oracle.ABSORB):
        np.testing.assert_array_equal(oracle.simulate(p, oracle.ASIAN_CALL, 16, 2, 0, 500, m), ref)


@pytest.mark.parametrize("mode", [oracle.PARTIAL_TRUNC, oracle.REFLECT])
def test_converges_to_analytic(mode):
    n = 200_000
    ref = analytic.heston_call(PB)
    r = oracle.simulate(PB, EC, 128, 23, 0, n, mode, threads=8)
    h = oracle.simulate(PB, EC, 64, 23, 0, n, mode, threads=8)
    m, se = oracle.mean_se(r[:, 3])
    m64, _ = oracle.mean_se(h[:, 3])
    assert abs(m - ref) < 3.5 * se + 2 * abs(m - m64)


@pytest.mark.parametrize("mode", [oracle.PARTIAL_TRUNC, oracle.REFLECT])
def test_martingale(mode):
    n = 200_000
    r = oracle.simulate(PB, EC, 32, 31, 0, n, mode, threads=8)
    m, se = oracle.mean_se(math.exp(-PB.r * PB.T) * r[:, 0])
    assert abs(m - PB.S0) < 4 * se
