"""Pins of the oracle's forward-mode derivatives under Andersen's QE scheme
(the paper's Future Work), the reference of the QE adjoint.

- The payoff column is the QE simulation's payoff, and d/dS0 and d/dr are the
  pathwise Delta and Rho of the same paths (S_T is S0 times a factor free of
  S0, and r enters the log-price additively as r t): exact identities.
- Central differences of the re-simulated payoff on the same Philox inputs,
  per path, for v0, kappa, theta, sigma and rho, at two step sizes: where the
  two agree the payoff is smooth between the bumps (no branch or payoff kink
  crossed), and there the derivative matches.  Paths whose branch margin is
  below the bump cannot be smooth; the test requires most paths to be.
- A small-vol-of-vol case where no step leaves the quadratic branch, at
  several step sizes, and a Feller-violating case where the exponential
  branch and its point mass at zero are taken.
"""
import numpy as np
import pytest

import oracle
from workloads import BASE

PB = oracle.Params(**BASE)
NAMES = ["S0", "v0", "r", "kappa", "theta", "sigma", "rho"]
CASES = {"base": PB, "feller-violated": PB.replace(sigma=0.9, kappa=1.0, theta=0.05),
         "low-vol-of-vol": PB.replace(sigma=0.1)}


@pytest.mark.parametrize("opt", [0, 1, 2, 3])
@pytest.mark.parametrize("case", list(CASES))
def test_qe_tangent_identities(opt, case):
    p = CASES[case]
    N, n = 24, 1500
    tan = oracle.tangent(p, opt, N, seed=5, n_paths=n, mode=oracle.QE, threads=8)
    rec = oracle.simulate(p, opt, N, seed=5, n_paths=n, mode=oracle.QE, threads=8)
    assert np.allclose(tan[:, 0], rec[:, 3], rtol=1e-14, atol=1e-14)
    assert np.allclose(tan[:, 1], rec[:, 4], rtol=1e-12, atol=1e-14)
    assert np.allclose(tan[:, 3], rec[:, 5], rtol=1e-11, atol=1e-11)
    m = oracle.simulate_qe(p, opt, N, 5, 0, n, threads=8)[1]
    assert np.array_equal(tan[:, 8], m)


@pytest.mark.parametrize("opt", [0, 2])
@pytest.mark.parametrize("case", list(CASES))
def test_qe_tangent_matches_finite_differences(opt, case):
    p = CASES[case]
    N, n = 24, 1500
    tan = oracle.tangent(p, opt, N, seed=12, n_paths=n, mode=oracle.QE, threads=8)
    for k, name in enumerate(NAMES):
        if name in ("S0", "r"):
            continue
        x0 = getattr(p, name)
        fds = []
        for h in (1e-5 * max(abs(x0), 0.1), 0.5e-5 * max(abs(x0), 0.1)):
            up = oracle.simulate(p.replace(**{name: x0 + h}), opt, N, seed=12, n_paths=n,
                                 mode=oracle.QE, threads=8)[:, 3]
            dn = oracle.simulate(p.replace(**{name: x0 - h}), opt, N, seed=12, n_paths=n,
                                 mode=oracle.QE, threads=8)[:, 3]
            fds.append((up - dn) / (2 * h))
        scale = np.maximum(np.abs(fds[1]), 1e-3 * np.abs(fds[1]).max() + 1e-12)
        smooth = np.abs(fds[0] - fds[1]) < 1e-6 * scale
        assert smooth.mean() > 0.9, (name, smooth.mean())
        err = np.abs(tan[smooth, 1 + k] - fds[1][smooth]) / scale[smooth]
        assert err.max() < 1e-5, (name, err.max(), int(np.argmax(err)))


def test_qe_tangent_branches_exercised():
    """The Feller-violating case takes the exponential branch, its point mass
    at zero and the quadratic branch; the low vol of vol case only the
    quadratic one."""
    p = CASES["feller-violated"]
    rec, margin, _ = oracle.simulate_qe(p, 0, 24, 5, 0, 1500, threads=8)
    assert (rec[:, 1] == 0).any() and (rec[:, 1] > 0).any()
    p = CASES["low-vol-of-vol"]
    zero = oracle.simulate_qe(p, 0, 24, 5, 0, 1500, threads=8)[0][:, 1] == 0
    assert not zero.any()


def test_qe_tangent_rejects_caller_normals():
    za = np.zeros((4, 3))
    with pytest.raises(ValueError):
        oracle.tangent(PB, 0, 3, n_paths=4, mode=oracle.QE, za=za, zb=za)
