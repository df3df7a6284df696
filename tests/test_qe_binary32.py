"""Why the single-precision QE parity bar is derived from binary32 evaluations.

The FP32 pricing kernel evaluates Andersen's QE scheme (the paper's Future
Work) in binary32.  ``tests/qe_binary32.py`` evaluates the same formulas, in
the kernel's scaled state and order, on the CPU.  These tests pin that
evaluation to the FP64 oracle, then show on the CPU that binary32 arithmetic
alone puts some QE paths further than 1e-5 from the oracle, by amounts that
grow with the path's amplification a_p of relative variance errors (reported
by the oracle), and that three times the spread of a 16-member
Monte-Carlo-arithmetic ensemble covers further independent binary32
evaluations.  The GPU QE parity tests use exactly that bar: per path and
column, max(1e-5 max(|oracle|, floor), 3 x ensemble spread).
"""
import numpy as np
import pytest

import oracle
from workloads import BASE

import qe_binary32 as qb

PB = oracle.Params(**BASE)
PF = PB.replace(kappa=0.5, theta=0.02, sigma=1.0, v0=0.02)  # Feller badly violated
U32 = 2.0 ** -24


def floors(p):
    return np.array([p.S0, max(p.v0, p.theta), p.S0, p.S0, 1.0, p.K * p.T])


def reference(p, t, N, seed, n, bumps):
    """Oracle records [n, 14] (bump columns from re-simulated scenarios), margins."""
    rec, margin, amp = oracle.simulate_qe(p, t, N, seed, 0, n, threads=8)
    ref = np.full((n, 14), np.nan)
    ref[:, :6] = rec
    if bumps:
        for k, (_, q) in enumerate(list(oracle.scenario_params(p, oracle.Bumps()).items())[1:]):
            r, m, _ = oracle.simulate_qe(q, t, N, seed, 0, n, threads=8)
            ref[:, 6 + k] = r[:, 3]
            margin = np.minimum(margin, m)
    return ref, margin, amp


@pytest.mark.parametrize("t", [0, 1, 2, 3, 4, 5])
@pytest.mark.parametrize("p", [PB, PF], ids=["feller", "high-vol-of-vol"])
def test_fp64_evaluation_equals_oracle(p, t):
    """In binary64 the kernel's formulation (scaled state, Taylor-series r
    bumps) gives the oracle's records: the module evaluates the oracle's
    arithmetic, so its binary32 deviations are rounding alone."""
    n, N = 1037, 13
    ref, _, _ = reference(p, t, N, 42, n, True)
    ev = qb.evaluate(p, t, N, 42, 0, n, bumps=True, dtype=np.float64)
    f = np.concatenate([floors(p), np.full(8, p.S0)])
    err = np.abs(ev - ref) / np.maximum(np.abs(ref), f)
    assert err.max() < 1e-11, (np.unravel_index(np.argmax(err), err.shape), err.max())


def test_binary32_misses_1e5_on_amplified_paths_only():
    """Round-to-nearest binary32: every path with a_p < 2 stays well inside
    1e-5; the terminal variance of an amplified path does not."""
    p, t, N, n, seed = PF, 0, 24, 4099, 7
    ref, margin, amp = reference(p, t, N, seed, n, False)
    ok = margin >= 1e-4
    err = np.abs(qb.evaluate(p, t, N, seed, 0, n)[:, :6] - ref[:, :6]) / np.maximum(
        np.abs(ref[:, :6]), floors(p))
    calm = ok & (amp < 2)
    assert calm.sum() > 2000
    assert err[calm].max() < 0.3e-5
    wild = ok & (amp >= 50)
    assert err[wild, 1].max() > 1e-5


@pytest.mark.parametrize("case", [(PF, 0, 24, 4099, 7), (PF, 2, 252, 1000, 7),
                                  (PB, 0, 24, 4099, 7)], ids=["pf-euro-24", "pf-asian-252",
                                                             "pb-euro-24"])
def test_binary32_error_scales_with_amplification(case):
    """Per path the binary32 error stays within 32 a_p roundings of every
    column, and the typical error of the log-price grows with a_p (the median
    at least doubles from a_p < 2 to a_p >= 10)."""
    p, t, N, n, seed = case
    ref, margin, amp = reference(p, t, N, seed, n, False)
    ok = margin >= 1e-4
    err = np.abs(qb.evaluate(p, t, N, seed, 0, n)[:, :6] - ref[:, :6]) / np.maximum(
        np.abs(ref[:, :6]), floors(p))
    assert (err[ok] <= 32 * U32 * amp[ok, None]).all()
    if p is PF:
        med = [np.median(err[ok & (amp >= lo) & (amp < hi), 0])
               for lo, hi in ((1, 2), (2, 10), (10, 1e9))]
        assert med[0] < med[1] < med[2] and med[2] > 2 * med[0], med


@pytest.mark.parametrize("case", [(PF, 2, 24, 4099, 7, True), (PF, 0, 252, 1000, 11, False),
                                  (PB, 2, 252, 1000, 3, False)],
                         ids=["pf-asian-24-bumps", "pf-euro-252", "pb-asian-252"])
def test_ensemble_bar_covers_other_binary32_evaluations(case):
    """Three times the spread of the 16-member ensemble (plus the
    round-to-nearest evaluation) bounds four further independent binary32
    evaluations on every path and column, with the 1e-5 floor."""
    p, t, N, n, seed, bumps = case
    ref, margin, _ = reference(p, t, N, seed, n, bumps)
    k = 14 if bumps else 6
    ref = ref[:, :k]
    ok = margin >= 1e-4
    f = np.concatenate([floors(p), np.full(8, p.S0)])[:k]
    bar = np.maximum(1e-5 * np.maximum(np.abs(ref), f),
                     3 * qb.spread(p, t, N, seed, 0, n, ref, bumps, members=16))
    for s in range(4):
        e = np.abs(qb.evaluate(p, t, N, seed, 0, n, bumps, rng=np.random.default_rng(500 + s))[:, :k]
                   - ref)
        assert (e[ok] <= bar[ok]).all(), s
