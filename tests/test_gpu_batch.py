"""GPU tests of the persistent batched kernel (heston_price_batch).

Each request of a batch is checked against the oracle's estimates on the same
paths, against its own result when priced alone (bitwise), and adjoint-mode
requests against the oracle's forward-mode derivatives.

FP64: relative 1e-10 on the sums.  FP32: the per-path bars of the parity
tests carried to the mean over the request's paths (sum of per-path bars / n):
1e-5 max(|o|, floor) for prices; for the pathwise Delta and Rho also the jump
of each path whose oracle average lies within ten times its own bar of the
strike (there the binary32 average may fall on the other side and switch the
indicator); for adjoint-mode payoffs and derivatives the per-path bars of the
adjoint parity tests, max(tol max(|o|, floor), 4 x spread), the spread being
how far Monte-Carlo-arithmetic evaluations in the kernel's precision land from
the oracle on the path (tests/tangent_binary32.py): where the variance comes
close to zero rounding alone moves a path's derivatives further than the
plain bar (tests/test_adjoint_conditioning.py).
"""
import numpy as np
import pytest

import oracle
import tangent_binary32 as tb
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
    out = {"price": oracle.mean_se(rec[:, 3]), "pw_delta": oracle.mean_se(rec[:, 4]),
           "pw_rho": oracle.mean_se(rec[:, 5])}
    return out, rec


def fp32_bars(q, rec):
    """Mean-level FP32 bars for price, pathwise Delta and Rho from the oracle's
    per-path records (see the module docstring)."""
    p = oracle.Params(**q["params"])
    n = rec.shape[0]
    X = rec[:, 2]
    D = np.exp(-p.r * p.T)
    near = np.abs(X - p.K) <= 10 * 1e-5 * np.maximum(np.abs(X), p.S0)
    jump_d = np.where(near, np.maximum(np.abs(rec[:, 4]), D * X / p.S0), 0.0)
    jump_r = np.where(near, np.maximum(np.abs(rec[:, 5]), D * p.T * np.maximum(X, p.K) * 1.01), 0.0)
    return {"price": (1e-5 * np.maximum(np.abs(rec[:, 3]), p.S0)).sum() / n,
            "pw_delta": (1e-5 * np.maximum(np.abs(rec[:, 4]), 1.0) + jump_d).sum() / n,
            "pw_rho": (1e-5 * np.maximum(np.abs(rec[:, 5]), p.K * p.T) + jump_r).sum() / n}


def adjoint_bars(q, prec):
    """Oracle tangent means [8] (price, 7 derivatives), their SEs and the
    mean-level bars (per-path bars summed over the paths / n)."""
    p = oracle.Params(**q["params"])
    tan = oracle.tangent(p, q["type"], q["n_steps"], q["seed"], 0, q["n_paths"], threads=8)
    per = tb.bars(p, q["type"], q["n_steps"], q["seed"], 0, q["n_paths"], tan,
                  dtype=np.float64 if prec == 0 else np.float32)
    m, se = oracle.mean_se(tan[:, :8])
    return m, se, per.mean(axis=0)


@pytest.mark.parametrize("scheme", [0, 1])
def test_batch_fp64_matches_oracle(hm, ctx, scheme):
    reqs = mixed_requests()
    res, _ = ctx.price_batch(reqs, hm.Options(precision=hm.FP64, scheme=scheme,
                                              greeks=hm.GREEKS_PATHWISE))
    for q, r in zip(reqs, res):
        ref, _ = oracle_estimates(q, oracle.ABSORB if scheme else oracle.FULL_TRUNC)
        for k in ("price", "pw_delta", "pw_rho"):
            assert r[k][0] == pytest.approx(ref[k][0], rel=1e-10, abs=1e-12), (q, k)
            assert r[k][1] == pytest.approx(ref[k][1], rel=1e-6, abs=1e-12), (q, k)
        assert r["n_paths"] == q["n_paths"]


def test_batch_fp32_matches_oracle(hm, ctx):
    reqs = mixed_requests()
    res, _ = ctx.price_batch(reqs, hm.Options(precision=hm.FP32, greeks=hm.GREEKS_PATHWISE))
    for q, r in zip(reqs, res):
        ref, rec = oracle_estimates(q)
        bar = fp32_bars(q, rec)
        for k in ("price", "pw_delta", "pw_rho"):
            assert abs(r[k][0] - ref[k][0]) <= bar[k], (q, k, r[k], ref[k], bar[k])


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
        m, se, bar = adjoint_bars(q, 0)
        assert r["price"][0] == pytest.approx(m[0], rel=1e-10, abs=1e-12)
        for k in range(7):
            assert abs(r["adj"][k][0] - m[1 + k]) <= bar[1 + k], (q, k)
            assert r["adj"][k][1] == pytest.approx(se[1 + k], rel=1e-4, abs=1e-12)


def serving_requests(n, seed=9, want=2):
    """Requests drawn as the serving workload's (Heston parameters as the
    portfolio's, many violating the Feller condition; 50..1000 steps), with
    path counts cut to a few thousand so the oracle finishes in seconds."""
    rs = workloads.request_stream(n, 1.0, seed=seed)
    return [dict(params=rs.params[i], type=int(rs.opt_type[i]), n_steps=int(rs.n_steps[i]),
                 n_paths=int(1000 + 317 * i), seed=int(rs.seed[i]), want=want)
            for i in range(n)]


def test_batch_fp32_adjoint_matches_oracle_derivatives(hm, ctx):
    """FP32 adjoint mode (the serving configuration) at 50..1000 steps."""
    reqs = serving_requests(8)
    assert min(q["n_steps"] for q in reqs) < 200 and max(q["n_steps"] for q in reqs) > 800
    res, _ = ctx.price_batch(reqs, hm.Options(precision=hm.FP32, greeks=hm.GREEKS_PATHWISE))
    for q, r in zip(reqs, res):
        m, se, bar = adjoint_bars(q, 1)
        assert abs(r["price"][0] - m[0]) <= bar[0], q
        for k in range(7):
            assert abs(r["adj"][k][0] - m[1 + k]) <= bar[1 + k], (q, k, r["adj"][k], m[1 + k])


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
    drawn per option; steps = ceil(252 T)) in one launch.  Checked against the
    oracle: the four options with the fewest path-steps, and the six
    longest-maturity options among those with at most 2^16 paths that violate
    the Feller condition (over a thousand FP32 steps each)."""
    pf = workloads.portfolio()
    reqs = [dict(params=pf.params(i), type=int(pf.opt_type[i]), n_steps=int(pf.n_steps[i]),
                 n_paths=int(pf.n_paths[i]), seed=int(pf.seed[i]), want=1) for i in range(len(pf))]
    res, ms = ctx.price_batch(reqs, hm.Options(precision=hm.FP32, greeks=hm.GREEKS_PATHWISE))
    assert all(np.isfinite(r["price"][0]) and r["price"][1] >= 0 for r in res)
    cost = pf.n_paths * pf.n_steps
    feller = 2 * pf.kappa * pf.theta < pf.sigma ** 2
    cand = np.nonzero((pf.n_paths <= 1 << 16) & feller)[0]
    long_ = cand[np.argsort(-pf.n_steps[cand])[:6]]
    assert len(long_) == 6 and pf.n_steps[long_].min() > 1000
    for i in list(np.argsort(cost)[:4]) + list(long_):
        ref, rec = oracle_estimates(reqs[i])
        bar = fp32_bars(reqs[i], rec)
        for k in ("price", "pw_delta", "pw_rho"):
            assert abs(res[i][k][0] - ref[k][0]) <= bar[k], (i, k, res[i][k], ref[k], bar[k])


def test_invalid_batch_requests(hm, ctx):
    good = mixed_requests()[:2]
    for bad in (dict(want=3), dict(n_paths=1), dict(type=7), dict(se_target=-1.0)):
        q = dict(good[0], **bad)
        with pytest.raises(hm.HestonError):
            ctx.price_batch([good[1], q])
    with pytest.raises(hm.HestonError):
        ctx.price_batch(good, hm.Options(fixings=(1, 2)))
    for scheme in (hm.EULER_FULL_TRUNCATION, hm.PARTIAL_TRUNCATION, hm.EXACT):
        with pytest.raises(hm.HestonError):
            ctx.price_batch(good, hm.Options(scheme=scheme))


# ---------------------------------------------------------------------------
# Andersen's QE scheme in the batched kernel (the paper's Future Work).  A QE
# path whose branch decision lies within the oracle's margin (column 8 of its
# QE tangent) can take the other branch in the kernel's arithmetic and then
# has an entirely different V'; the mean-level bars cannot absorb that, so
# the oracle comparisons use requests with no path within 1e-9 (FP64) or
# 1e-4 (FP32) of a branch switch, which each test checks; bitwise alone/mix
# agreement (and, in tests/test_gpu_server.py, served/batch agreement) covers
# all requests.

def qe_margin(q):
    p = oracle.Params(**q["params"])
    return oracle.simulate_qe(p, q["type"], q["n_steps"], q["seed"], 0, q["n_paths"],
                              threads=8)[1]


def qe_clear(reqs, thr):
    return [q for q in reqs if qe_margin(q).min() >= thr]


def test_batch_qe_fp64_matches_oracle(hm, ctx):
    reqs = qe_clear(mixed_requests(), 1e-9)
    assert len(reqs) >= 8
    res, _ = ctx.price_batch(reqs, hm.Options(precision=hm.FP64, scheme=hm.QE,
                                              greeks=hm.GREEKS_PATHWISE))
    for q, r in zip(reqs, res):
        ref, _ = oracle_estimates(q, oracle.QE)
        for k in ("price", "pw_delta", "pw_rho"):
            assert r[k][0] == pytest.approx(ref[k][0], rel=1e-10, abs=1e-12), (q, k)
            assert r[k][1] == pytest.approx(ref[k][1], rel=1e-6, abs=1e-12), (q, k)


def qe_adjoint_bars(q, prec):
    p = oracle.Params(**q["params"])
    tan = oracle.tangent(p, q["type"], q["n_steps"], q["seed"], 0, q["n_paths"], oracle.QE,
                         threads=8)
    per = tb.bars(p, q["type"], q["n_steps"], q["seed"], 0, q["n_paths"], tan, oracle.QE,
                  dtype=np.float64 if prec == 0 else np.float32)
    m, se = oracle.mean_se(tan[:, :8])
    return m, se, per.mean(axis=0), tan[:, 8]


def test_batch_qe_adjoint_fp64_matches_oracle(hm, ctx):
    reqs = mixed_requests(want=hm.WANT_ADJOINT)
    res, _ = ctx.price_batch(reqs, hm.Options(precision=hm.FP64, scheme=hm.QE,
                                              greeks=hm.GREEKS_PATHWISE))
    checked = 0
    for q, r in zip(reqs, res):
        m, se, bar, margin = qe_adjoint_bars(q, 0)
        if margin.min() < 1e-9:
            continue
        checked += 1
        assert r["price"][0] == pytest.approx(m[0], rel=1e-10, abs=1e-12)
        for k in range(7):
            assert abs(r["adj"][k][0] - m[1 + k]) <= bar[1 + k], (q, k)
            assert r["adj"][k][1] == pytest.approx(se[1 + k], rel=1e-4, abs=1e-12)
    assert checked >= 8


def qe_fp32_requests(n=6, want=2):
    """Requests at the base parameters (Feller holds, so no QE step comes near
    a branch switch), 50..400 steps, every option type."""
    g = np.random.default_rng(13)
    base = dict(workloads.BASE)
    out = []
    for i in range(n):
        p = dict(base, K=float(g.uniform(85, 115)), T=float(g.uniform(0.5, 2.0)))
        out.append(dict(params=p, type=i % 4, n_steps=int(g.integers(50, 401)),
                        n_paths=int(1500 + 611 * i), seed=int(g.integers(0, 2**62)), want=want))
    return out


def test_batch_qe_fp32_adjoint_matches_oracle(hm, ctx):
    reqs = qe_fp32_requests()
    res, _ = ctx.price_batch(reqs, hm.Options(precision=hm.FP32, scheme=hm.QE,
                                              greeks=hm.GREEKS_PATHWISE))
    for q, r in zip(reqs, res):
        m, se, bar, margin = qe_adjoint_bars(q, 1)
        assert margin.min() >= 1e-4, q
        assert abs(r["price"][0] - m[0]) <= bar[0], q
        for k in range(7):
            assert abs(r["adj"][k][0] - m[1 + k]) <= bar[1 + k], (q, k, r["adj"][k], m[1 + k])


def test_batch_qe_fp32_price_mode_matches_oracle(hm, ctx):
    """Price mode: the price and the pathwise Delta and Rho (the tangent's
    d/dS0 and d/dr) within the same mean-level bars."""
    reqs = qe_fp32_requests(want=1)
    res, _ = ctx.price_batch(reqs, hm.Options(precision=hm.FP32, scheme=hm.QE,
                                              greeks=hm.GREEKS_PATHWISE))
    for q, r in zip(reqs, res):
        m, se, bar, margin = qe_adjoint_bars(q, 1)
        assert margin.min() >= 1e-4, q
        for k, col in (("price", 0), ("pw_delta", 1), ("pw_rho", 3)):
            assert abs(r[k][0] - m[col]) <= bar[col], (q, k, r[k], m[col], bar[col])


@pytest.mark.parametrize("want", [1, 2])
def test_batch_qe_alone_and_in_the_mix_are_bitwise_equal(hm, ctx, want):
    reqs = mixed_requests(want=want)
    opts = hm.Options(precision=hm.FP32, scheme=hm.QE, greeks=hm.GREEKS_PATHWISE)
    mix, _ = ctx.price_batch(reqs, opts)
    for i in (1, 4, 10):
        alone, _ = ctx.price_batch([reqs[i]], opts)
        for k in ("price", "pw_delta", "pw_rho", "adj"):
            assert alone[0][k] == mix[i][k], (i, k)
