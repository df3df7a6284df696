"""Pins of the oracle's Euler modes (paper, Background, "Euler
discretisation"): the Milstein steps without the Milstein term, with either
truncation.  Facts outside the oracle: the paper's statement that the two
schemes differ by the term sigma^2 dt (Z2^2 - 1) / 4 in the variance step
(checked on the pinned Philox normals), the identity of the schemes when that
term vanishes (sigma = 0), the characteristic-function price, the martingale.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import analytic
from workloads import BASE

PB = oracle.Params(**BASE)
EC = oracle.EURO_CALL
EULER = {oracle.FULL_TRUNC: oracle.EULER_FULL_TRUNC, oracle.ABSORB: oracle.EULER_ABSORB}


@pytest.mark.parametrize("mode", [oracle.FULL_TRUNC, oracle.ABSORB])
def test_one_step_differs_from_milstein_by_the_milstein_term(mode):
    n = 4000
    za, zb = oracle.normals(13, 0, n, 1)
    z2 = PB.rho * za[:, 0] + math.sqrt(1 - PB.rho ** 2) * zb[:, 0]
    mil = oracle.simulate(PB, EC, 1, 13, 0, n, mode)
    eul = oracle.simulate(PB, EC, 1, 13, 0, n, EULER[mode])
    np.testing.assert_array_equal(mil[:, 0], eul[:, 0])  # the price step has no such term
    term = 0.25 * PB.sigma ** 2 * PB.T * (z2 ** 2 - 1.0)
    if mode == oracle.FULL_TRUNC:
        np.testing.assert_allclose(mil[:, 1] - eul[:, 1], term, rtol=0, atol=1e-15)
    else:  # absorption clamps both at zero afterwards
        pos = (mil[:, 1] > 0) & (eul[:, 1] > 0)
        assert pos.mean() > 0.5
        np.testing.assert_allclose(mil[pos, 1] - eul[pos, 1], term[pos], rtol=0, atol=1e-15)


def test_euler_equals_milstein_without_vol_of_vol():
    p = PB.replace(sigma=0.0)
    a = oracle.simulate(p, oracle.ASIAN_CALL, 24, 3, 0, 500)
    b = oracle.simulate(p, oracle.ASIAN_CALL, 24, 3, 0, 500, oracle.EULER_FULL_TRUNC)
    np.testing.assert_array_equal(a, b)


@pytest.mark.parametrize("mode", [oracle.EULER_FULL_TRUNC, oracle.EULER_ABSORB])
def test_euler_european_matches_analytic(mode):
    n = 200_000
    ref = analytic.heston_call(PB)
    r = oracle.simulate(PB, EC, 128, 17, 0, n, mode, threads=8)
    h = oracle.simulate(PB, EC, 64, 17, 0, n, mode, threads=8)
    m, se = oracle.mean_se(r[:, 3])
    m64, _ = oracle.mean_se(h[:, 3])
    assert abs(m - ref) < 3.5 * se + 2 * abs(m - m64)


def test_euler_martingale():
    n = 200_000
    r = oracle.simulate(PB, EC, 32, 29, 0, n, oracle.EULER_FULL_TRUNC, threads=8)
    m, se = oracle.mean_se(math.exp(-PB.r * PB.T) * r[:, 0])
    assert abs(m - PB.S0) < 4 * se


def test_euler_truncations():
    """Absorption keeps every variance >= 0 (the paper's max(V, 0) after each
    step); full truncation carries negative values."""
    p = PB.replace(sigma=0.8, kappa=1.0, theta=0.02, v0=0.02)
    a = oracle.simulate(p, EC, 16, 8, 0, 4000, oracle.EULER_ABSORB)
    f = oracle.simulate(p, EC, 16, 8, 0, 4000, oracle.EULER_FULL_TRUNC)
    assert (a[:, 1] >= 0).all()
    assert (f[:, 1] < 0).mean() > 0.05
