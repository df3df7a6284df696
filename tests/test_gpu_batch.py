"""GPU tests of the persistent batched kernel (heston_price_batch).

Each request of a batch is checked against the oracle's estimates on the same
paths (FP64: relative 1e-10 on the sums; FP32: the per-path bar 1e-5 S0
carried to the mean), against its own result when priced alone (bitwise), and
adjoint-mode requests against the oracle's forward-mode derivatives.
"""
import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu


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


def mixed_requests(want=1):
    g = np.random.default_rng(7)
    reqs = []
    for i in range(12):
        p = dict(S0=100.0, K=float(g.uniform(80, 120)), r=0.05, T=float(g.uniform(0.2, 2.0)),
                 v0=float(g.uniform(0.01, 0.09)), kappa=float(g.uniform(0.5, 4.0)),
                 theta=float(g.uniform(0.01, 0.09)), sigma=float(g.uniform(0.1, 0.8)),
                 rho=float(g.uniform(-0.9, 0.0)))
        reqs.append(dict(params=p, type=i % 4, n_steps=int(g.integers(1, 60)),
                         n_paths=[1000, 1025, 3000, 2048, 17, 4096 + 3][i % 6],
                         seed=int(g.integers(0, 2**63)), want=want))
    return reqs


def oracle_estimates(q, mode=oracle.FULL_TRUNC):
    p = oracle.Params(**q["params"])
    rec = oracle.simulate(p, q["type"], q["n_steps"], q["seed"], 0, q["n_paths"], mode,
                          threads=8)
    return {"price": oracle.mean_se(rec[:, 3]), "pw_delta": oracle.mean_se(rec[:, 4]),
            "pw_rho": oracle.mean_se(rec[:, 5])}


@pytest.mark.parametrize("scheme", [0, 1])
def test_batch_fp64_matches_oracle(hm, ctx, scheme):
    reqs = mixed_requests()
    res, _ = ctx.price_batch(reqs, hm.Options(precision=hm.FP64, scheme=scheme,
                                              greeks=hm.GREEKS_PATHWISE))
    for q, r in zip(reqs, res):
        ref = oracle_estimates(q, oracle.ABSORB if scheme else oracle.FULL_TRUNC)
        for k in ("price", "pw_delta", "pw_rho"):
            assert r[k][0] == pytest.approx(ref[k][0], rel=1e-10, abs=1e-12), (q, k)
            assert r[k][1] == pytest.approx(ref[k][1], rel=1e-6, abs=1e-12), (q, k)
        assert r["n_paths"] == q["n_paths"]


def test_batch_fp32_matches_oracle(hm, ctx):
    reqs = mixed_requests()
    res, _ = ctx.price_batch(reqs, hm.Options(precision=hm.FP32, greeks=hm.GREEKS_PATHWISE))
    for q, r in zip(reqs, res):
        ref = oracle_estimates(q)
        assert abs(r["price"][0] - ref["price"][0]) <= 1e-5 * q["params"]["S0"], q
        # pathwise indicators may flip only on paths within 1e3 tol K of the strike
        assert abs(r["pw_delta"][0] - ref["pw_delta"][0]) <= 1e-5 + 0.02, q


def test_alone_and_in_the_mix_are_bitwise_equal(hm, ctx):
    reqs = mixed_requests()
    opts = hm.Options(precision=hm.FP32, greeks=hm.GREEKS_PATHWISE)
    mix, _ = ctx.price_batch(reqs, opts)
    for i in (0, 3, 7, 11):
        alone, _ = ctx.price_batch([reqs[i]], opts)
        for k in ("price", "pw_delta", "pw_rho"):
            assert alone[0][k] == mix[i][k], (i, k)
    # and a batch in reverse order
    rev, _ = ctx.price_batch(reqs[::-1], opts)
    for i, r in enumerate(rev[::-1]):
        assert r["price"] == mix[i]["price"]


def test_batch_adjoint_matches_oracle_derivatives(hm, ctx):
    reqs = mixed_requests(want=hm.WANT_ADJOINT)
    res, _ = ctx.price_batch(reqs, hm.Options(precision=hm.FP64, greeks=hm.GREEKS_PATHWISE))
    for q, r in zip(reqs, res):
        p = oracle.Params(**q["params"])
        tan = oracle.tangent(p, q["type"], q["n_steps"], q["seed"], 0, q["n_paths"], threads=8)
        m, se = oracle.mean_se(tan[:, :8])
        assert r["price"][0] == pytest.approx(m[0], rel=1e-10, abs=1e-12)
        # per-path bar tol max(|o|, floor) max(1, a_p) (as for the standalone
        # adjoint), carried to the mean of the paths
        amp = np.maximum(1.0, tan[:, 8])
        floors = [1.0, p.S0, p.K * p.T, p.S0 * p.T, p.S0 * p.T, p.S0, p.S0]
        for k in range(7):
            bound = (1e-12 * np.maximum(np.abs(tan[:, 1 + k]), floors[k]) * amp).mean()
            assert abs(r["adj"][k][0] - m[1 + k]) <= bound, (q, k)
            assert r["adj"][k][1] == pytest.approx(se[1 + k], rel=1e-4, abs=1e-12)


def test_mixed_modes_in_one_batch(hm, ctx):
    a = mixed_requests(want=hm.WANT_PATHWISE)[:6]
    b = mixed_requests(want=hm.WANT_ADJOINT)[6:]
    opts = hm.Options(precision=hm.FP32, greeks=hm.GREEKS_PATHWISE)
    mix, _ = ctx.price_batch(a + b, opts)
    ra, _ = ctx.price_batch(a, opts)
    rb, _ = ctx.price_batch(b, opts)
    for x, y in zip(mix, ra + rb):
        assert x["price"] == y["price"]
        assert x["adj"] == y["adj"]


def test_portfolio_4096_options(hm, ctx):
    """The 4096-option portfolio (K, T, paths 2^14..2^20, Heston parameters
    drawn per option; steps = ceil(252 T)) in one launch; the six options with
    the fewest path-steps are checked against the oracle."""
    pf = workloads.portfolio()
    reqs = [dict(params=pf.params(i), type=int(pf.opt_type[i]), n_steps=int(pf.n_steps[i]),
                 n_paths=int(pf.n_paths[i]), seed=int(pf.seed[i]), want=1) for i in range(len(pf))]
    res, ms = ctx.price_batch(reqs, hm.Options(precision=hm.FP32, greeks=hm.GREEKS_PATHWISE))
    assert all(np.isfinite(r["price"][0]) and r["price"][1] >= 0 for r in res)
    cost = pf.n_paths * pf.n_steps
    for i in np.argsort(cost)[:6]:
        ref = oracle_estimates(reqs[i])
        assert abs(res[i]["price"][0] - ref["price"][0]) <= 1e-5 * 100.0, (i, res[i], ref)


def test_invalid_batch_requests(hm, ctx):
    good = mixed_requests()[:2]
    for bad in (dict(want=3), dict(n_paths=1), dict(type=7), dict(se_target=-1.0)):
        q = dict(good[0], **bad)
        with pytest.raises(hm.HestonError):
            ctx.price_batch([good[1], q])
    with pytest.raises(hm.HestonError):
        ctx.price_batch(good, hm.Options(fixings=(1, 2)))
