"""heston_price_greeks_noalloc (the entry point for callers that cannot
allocate) against heston_price_greeks_ex: two calls in a row on one device,
the second with a smaller input, each bitwise equal to the context call with
the same arguments (same kernels, same launch shape, same reduction order).
"""
import ctypes

import numpy as np
import pytest

import oracle
from workloads import BASE

pytestmark = pytest.mark.gpu

KEYS = ("price", "pw_delta", "pw_rho", "delta", "gamma", "vega", "rho", "theta")


@pytest.fixture(scope="module")
def hm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2309_10477_amd as hm
    hm.lib()
    return hm


@pytest.fixture(scope="module")
def ctx(hm):
    c = hm.Context(0)
    yield c
    c.close()


def same(a, b):
    for k in KEYS:
        assert a[k] == b[k], (k, a[k], b[k])
    assert a["n_paths"] == b["n_paths"] and a["valid_mask"] == b["valid_mask"]


def test_two_calls_match_the_context_call(hm, ctx):
    import torch
    print("noalloc: FP32 Asian 2^18 x 252 fused bumps, then FP64 European 5003 x 40", flush=True)
    cases = [
        (hm.ASIAN_CALL, 1 << 18, 252, 42, hm.Options(precision=hm.FP32)),
        (hm.EURO_PUT, 5003, 40, 7, hm.Options(precision=hm.FP64)),
    ]
    for t, n, N, seed, o in cases:
        a = hm.price_greeks_noalloc(BASE, t, n, N, seed, o)
        torch.cuda.synchronize()
        b = ctx.price_greeks(BASE, t, n, N, seed, o)
        same(a, b)
        assert a["device_ms"] > 0 and a["latency_ms"] >= a["device_ms"]


def test_fixings_schemes_and_streams(hm, ctx):
    import torch
    print("noalloc: quarterly fixings, QE, absorption, on a torch stream", flush=True)
    s = torch.cuda.Stream()
    cases = [
        (hm.ASIAN_PUT, 40_000, 200, 3, hm.Options(precision=hm.FP64, fixings=(50, 100, 150, 200))),
        (hm.ASIAN_CALL, 20_000, 64, 4, hm.Options(precision=hm.FP32, scheme=hm.QE)),
        (hm.EURO_CALL, 3_000, 16, 5, hm.Options(precision=hm.FP32, scheme=hm.ABSORPTION,
                                                greeks=hm.GREEKS_PATHWISE)),
    ]
    for t, n, N, seed, o in cases:
        a = hm.price_greeks_noalloc(BASE, t, n, N, seed, o, stream=s)
        b = ctx.price_greeks(BASE, t, n, N, seed, o)
        same(a, b)


def test_matches_oracle_fp64(hm):
    """Small FP64 case against the oracle's estimates (the parity bar of the
    summed estimators, 1e-10 relative)."""
    n, N, seed = 10_000, 100, 42
    r = hm.price_greeks_noalloc(BASE, hm.EURO_CALL, n, N, seed, hm.Options(precision=hm.FP64))
    ref = oracle.price_greeks(oracle.Params(**BASE), oracle.EURO_CALL, n, N, seed, threads=8)
    for k in ("price", "pw_delta", "delta", "vega", "rho", "theta"):
        assert r[k][0] == pytest.approx(ref[k][0], rel=1e-10, abs=1e-11), k


def test_rejects_what_does_not_fit(hm):
    print("noalloc: size and option rejections", flush=True)
    with pytest.raises(hm.HestonError, match="bytes of device scratch"):
        hm.price_greeks_noalloc(BASE, hm.EURO_CALL, 1 << 26, 10, 1, hm.Options(precision=hm.FP32))
    with pytest.raises(hm.HestonError):
        hm.price_greeks_noalloc(BASE, hm.EURO_CALL, 1 << 16, 10, 1,
                                hm.Options(precision=hm.FP32, rng=hm.SOBOL_BRIDGE))
    # a rejected call leaves the next one intact
    r = hm.price_greeks_noalloc(BASE, hm.EURO_CALL, 4096, 10, 1, hm.Options(precision=hm.FP64))
    assert np.isfinite(r["price"][0])
