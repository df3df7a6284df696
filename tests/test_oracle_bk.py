"""Pins of the oracle's Broadie-Kaya exact simulator (no GPU needed).

Paper: algorithm "Broadie and Kaya exact simulation algorithm" and the two
bottleneck sections (V_t given V_u; the integral of V given both ends).
"""
import json
import math
import os

import numpy as np
import pytest
from scipy import stats

import oracle
from oracle import analytic, bk
from workloads import PAPER

HERE = os.path.dirname(os.path.abspath(__file__))
GOLD = json.load(open(os.path.join(HERE, "golden", "paper_values.json")))
PP = oracle.Params(**PAPER)


@pytest.mark.parametrize("p", [PP, PP.replace(theta=0.004, sigma=0.7)])
def test_variance_transition_is_scaled_noncentral_chi2(p):
    """V_t / c against scipy's non-central chi-square (KS), both for d > 1 (the
    paper's decomposition) and d <= 1 (Poisson mixture)."""
    dt, vu = 0.25, 0.02
    rng = np.random.Generator(np.random.PCG64(3))
    x = bk.sample_vt(p, np.full(40000, vu), dt, rng)
    e = math.exp(-p.kappa * dt)
    c = p.sigma ** 2 * (1 - e) / (4 * p.kappa)
    d = 4 * p.kappa * p.theta / p.sigma ** 2
    lam = vu * e / c
    assert stats.kstest(x / c, stats.ncx2(d, lam).cdf).pvalue > 1e-3
    # conditional mean of the CIR process
    m = p.theta + (vu - p.theta) * e
    assert abs(x.mean() - m) < 4 * x.std() / math.sqrt(x.size)


@pytest.mark.parametrize("vu,vt", [(0.010201, 0.02), (0.010201, 0.001), (0.05, 0.03)])
def test_integrated_variance_cdf(vu, vt):
    iv = bk.IntegratedVariance(PP, 1.0)
    h, ueps, rp = iv.cdf_grid(vu, vt)
    xs = np.linspace(0.0, ueps, 4001)
    F = np.array([iv.cdf(x, h, rp) for x in xs])
    assert F[0] == 0.0 and abs(F[-1] - 1.0) < 1e-8
    assert np.all(np.diff(F) > -1e-9)
    mean_from_cdf = np.trapezoid(1.0 - F, xs)
    # two numerical routes to the conditional mean: the CDF integral and the slope of Phi at 0
    assert mean_from_cdf == pytest.approx(iv.moments(vu, vt)[0], rel=1e-5)
    for u in (1e-4, 0.3, 0.9, 0.9999):
        x = iv.sample(vu, vt, u)
        assert iv.cdf(x, h, rp) == pytest.approx(u, abs=1e-11)


def test_integrated_variance_unconditional_mean():
    """E[int_0^D V] = theta D + (v0 - theta)(1 - e^{-kappa D})/kappa, averaging the
    conditional draws over V_D drawn from its transition law."""
    p, D, n = PP, 0.5, 3000
    rng = np.random.Generator(np.random.PCG64(9))
    vt = bk.sample_vt(p, np.full(n, p.v0), D, rng)
    iv = bk.IntegratedVariance(p, D)
    I = np.array([iv.sample(p.v0, v, u) for v, u in zip(vt, rng.uniform(size=n))])
    ref = p.theta * D + (p.v0 - p.theta) * (1 - math.exp(-p.kappa * D)) / p.kappa
    assert abs(I.mean() - ref) < 4 * I.std() / math.sqrt(n)


@pytest.mark.slow
def test_bk_european_matches_characteristic_function():
    v, se = bk.price(PP, False, 6000, seed=11)
    assert abs(v - analytic.heston_call(PP)) < 3.5 * se


@pytest.mark.slow
def test_bk_asian_matches_paper_exact_simulation():
    """Quarterly fixings: the paper's exact-simulation QMC value 4.3840 (0.0064)."""
    g = GOLD["asian_bk_qmc_512"]
    v, se = bk.price(PP, True, 3000, seed=12, times=g["fixing_times"])
    assert abs(v - g["value"]) < 3.5 * math.hypot(se, g["std"])


@pytest.mark.parametrize("asian", [False, True], ids=["european", "asian"])
def test_bk_reproduces_paper_mc_columns(asian):
    """The Monte-Carlo column of the paper's exact-simulation tables (64 to 2048
    paths; 30-run mean and std), one control-variate run per row within 4
    combined errors."""
    tab = GOLD["exact_asian_mc" if asian else "exact_european_mc"]
    times = GOLD["asian_bk_qmc_512"]["fixing_times"] if asian else None
    for n, val, std in zip(tab["paths"], tab["value"], tab["std"]):
        v, se = bk.price(PP, asian, n, seed=4000 + n, times=times)
        assert abs(v - val) < 4 * math.hypot(se, std), (n, v, se, val, std)
