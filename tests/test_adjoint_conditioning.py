"""Why the adjoint parity bars grow where the variance nears zero.

The GPU adjoint tests compare per-path derivatives with the oracle's
forward-mode derivatives under tol max(|oracle|, floor) max(1, a_p), a_p the
path's largest d sqrt(V+ dt)/dV+ = sqrt(dt/V+)/2; in FP32 at parameters that
violate the Feller condition the allowance is the rounding spread measured by
``tests/tangent_spread.py``.  These CPU tests show, on the oracle alone, what
those bars rest on: perturbing every step's normals by one rounding moves the
oracle's own derivatives by more than the plain bar on paths with large a_p,
by less than the a_p-scaled bar everywhere in binary64, and in binary32 at
Feller-violating parameters by far more than even the a_p-scaled bar.
"""
import numpy as np
import pytest

import oracle
import workloads
from workloads import BASE

import tangent_spread as ts

PB = oracle.Params(**BASE)


def floors(p):
    return np.array([p.S0, 1.0, p.S0, p.K * p.T, p.S0 * p.T, p.S0 * p.T, p.S0, p.S0])


def test_fp64_spread_needs_and_fits_the_amplified_bar():
    """Vol of vol 0.6 (the FP64 adjoint parity case): one-rounding
    perturbations exceed 1e-12 relative on amplified paths, and stay inside
    1e-12 max(1, a_p) on every path."""
    p, N, n = PB.replace(sigma=0.6), 37, 2013
    tan, s = ts.spread(p, 0, N, 11, 0, n, 0, ulps=1.0)
    amp = np.maximum(1.0, tan[:, 8])
    rel = s / np.maximum(np.abs(tan[:, :8]), floors(p))
    assert amp.max() > 100
    assert rel[amp > 50].max() > 1e-12
    assert (rel <= 1e-12 * amp[:, None]).all()
    # and the sensitivity grows with a_p
    med = [np.median(rel[(amp >= lo) & (amp < hi), 2]) for lo, hi in ((1, 5), (5, 50), (50, 1e9))]
    assert med[0] < med[1] < med[2]


def test_fp32_spread_at_the_base_parameters_fits_the_plain_bar():
    """The FP32 adjoint parity case (Feller satisfied, a_p below 3): four-rounding
    binary32 perturbations stay far inside 1e-5 max(1, a_p)."""
    tan, s = ts.spread(PB, 0, 100, 5, 0, 4196, 1)
    amp = np.maximum(1.0, tan[:, 8])
    assert amp.max() < 3
    assert (s / np.maximum(np.abs(tan[:, :8]), floors(PB)) <= 0.2e-5 * amp[:, None]).all()


def test_fp32_spread_without_feller_exceeds_even_the_amplified_bar():
    """A serving-workload request that violates the Feller condition
    (2 kappa theta / sigma^2 = 0.11): binary32-sized perturbations move some
    paths' derivatives by more than 1e-5 max(|o|, floor) max(1, a_p), so FP32
    parity there can only be judged against the measured spread."""
    rs = workloads.request_stream(12, 1.0, seed=9)
    i = 11
    p = oracle.Params(**rs.params[i])
    assert 2 * p.kappa * p.theta / p.sigma ** 2 < 0.2
    tan, s = ts.spread(p, int(rs.opt_type[i]), int(rs.n_steps[i]), int(rs.seed[i]), 0, 2048, 1,
                       members=4)
    amp = np.maximum(1.0, tan[:, 8])
    bar = 1e-5 * np.maximum(np.abs(tan[:, :8]), floors(p)) * amp[:, None]
    assert (s > bar).any()
