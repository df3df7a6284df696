"""GPU tests of the continuous-batching request loop (heston_server_*).

A served request's result must be the same alone and in a mix of concurrent
requests (bitwise: its items and their fold order do not depend on the mix),
agree with the batch API and the oracle on the same paths, stop at the first
item boundary where the price SE meets its target, and come through a tiny
memory budget that forces requests to wait for admission.
"""
import math
import time

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


def requests(n, want=1, se_target=0.0, seed=11):
    g = np.random.default_rng(seed)
    out = []
    for i in range(n):
        p = dict(S0=100.0, K=float(g.uniform(80, 120)), r=0.05, T=float(g.uniform(0.2, 2.0)),
                 v0=float(g.uniform(0.01, 0.09)), kappa=float(g.uniform(0.5, 4.0)),
                 theta=float(g.uniform(0.01, 0.09)), sigma=float(g.uniform(0.1, 0.8)),
                 rho=float(g.uniform(-0.9, 0.0)))
        out.append(dict(params=p, type=int(g.integers(0, 4)), n_steps=int(g.integers(5, 80)),
                        n_paths=int(g.integers(1000, 40000)), seed=int(g.integers(0, 2**62)),
                        want=want, se_target=se_target))
    return out


def serve(hm, ctx, reqs, **cfg):
    srv = hm.Server(ctx, **cfg)
    try:
        tickets = [srv.submit(**q) for q in reqs]
        res = [srv.wait(t, 120_000) for t in tickets]
        stats = srv.stats()
    finally:
        srv.close()
    assert all(r is not None for r in res)
    return res, stats


@pytest.mark.parametrize("want", [1, 2])
def test_alone_and_in_the_mix(hm, ctx, want):
    reqs = requests(24, want=want)
    mix, stats = serve(hm, ctx, reqs, precision=hm.FP32)
    assert stats["completed"] == 24 and stats["p50_ms"] > 0 and stats["p99_ms"] >= stats["p50_ms"]
    # latency: submit to completion; device time: the launches that carried its items
    lat = np.array([r["latency_ms"] for r in mix])
    # the server's percentiles are nearest-rank: the ceil(q n)-th smallest latency
    rank50 = np.sort(lat)[math.ceil(0.5 * lat.size) - 1]
    assert (lat > 0).all() and stats["p50_ms"] == pytest.approx(rank50, rel=1e-9)
    # device time sums the durations of the launches that carried the request's
    # items; at most three launches (the engine's launch slots) are in flight at
    # once, so the sum is at most three times the request's wall latency
    assert all(0 < r["device_ms"] <= 3 * r["latency_ms"] for r in mix)
    for i in (0, 5, 17):
        alone, _ = serve(hm, ctx, [reqs[i]], precision=hm.FP32)
        for k in ("price", "pw_delta", "pw_rho", "adj", "n_paths"):
            assert alone[0][k] == mix[i][k], (i, k)


def test_served_fp64_matches_batch_and_oracle(hm, ctx):
    reqs = requests(10)
    res, _ = serve(hm, ctx, reqs, precision=hm.FP64)
    bat, _ = ctx.price_batch(reqs, hm.Options(precision=hm.FP64, greeks=hm.GREEKS_PATHWISE))
    for q, r, b in zip(reqs, res, bat):
        assert r["n_paths"] == q["n_paths"]
        for k in ("price", "pw_delta", "pw_rho"):
            assert r[k][0] == pytest.approx(b[k][0], rel=1e-12, abs=1e-13)
        p = oracle.Params(**q["params"])
        rec = oracle.simulate(p, q["type"], q["n_steps"], q["seed"], 0, q["n_paths"], threads=8)
        m, se = oracle.mean_se(rec[:, 3])
        assert r["price"][0] == pytest.approx(m, rel=1e-10, abs=1e-12)
        assert r["price"][1] == pytest.approx(se, rel=1e-6)


def test_served_fp32_adjoint_matches_oracle(hm, ctx):
    """Served requests in the serving workload's mode (FP32, adjoint
    sensitivities, 50..1000 steps, Heston parameters of the request stream)
    against the oracle's forward-mode derivatives on the same paths, with the
    mean-level bars of the batch tests: per path max(1e-5 max(|o|, floor),
    4 x the binary32 spread of tests/tangent_binary32.py), summed over the
    paths / n."""
    rs = workloads.request_stream(6, 1.0, seed=21)
    reqs = [dict(params=rs.params[i], type=int(rs.opt_type[i]), n_steps=int(rs.n_steps[i]),
                 n_paths=2048 + 999 * i, seed=int(rs.seed[i]), want=2) for i in range(6)]
    assert max(q["n_steps"] for q in reqs) > 300
    res, _ = serve(hm, ctx, reqs, precision=hm.FP32)
    for q, r in zip(reqs, res):
        assert r["n_paths"] == q["n_paths"]
        p = oracle.Params(**q["params"])
        tan = oracle.tangent(p, q["type"], q["n_steps"], q["seed"], 0, q["n_paths"], threads=8)
        bar = tb.bars(p, q["type"], q["n_steps"], q["seed"], 0, q["n_paths"], tan).mean(axis=0)
        m = tan[:, :8].mean(axis=0)
        assert abs(r["price"][0] - m[0]) <= bar[0], q
        for k in range(7):
            assert abs(r["adj"][k][0] - m[1 + k]) <= bar[1 + k], (q, k, r["adj"][k], m[1 + k])


def test_se_target_stops_at_first_item_boundary(hm, ctx):
    reqs = requests(8, se_target=0.25, seed=5)
    for q in reqs:
        q["n_paths"] = 1 << 20
    res, _ = serve(hm, ctx, reqs, precision=hm.FP64)
    for q, r in zip(reqs, res):
        n = r["n_paths"]
        assert n % 1024 == 0 and n >= 2048
        assert r["price"][1] <= 0.25
        p = oracle.Params(**q["params"])
        rec = oracle.simulate(p, q["type"], q["n_steps"], q["seed"], 0, n, threads=8)
        m, se = oracle.mean_se(rec[:, 3])
        assert r["price"][0] == pytest.approx(m, rel=1e-10, abs=1e-12)
        if n > 2048:  # one item fewer would not have met the target
            assert oracle.mean_se(rec[: n - 1024, 3])[1] > 0.25


def test_tiny_budget_queues_but_completes(hm, ctx):
    """A budget whose request pool holds about three request states: the rest
    wait in the queue and are admitted as earlier ones finish; results are
    bitwise those of an unconstrained server."""
    reqs = requests(12)
    big, _ = serve(hm, ctx, reqs, precision=hm.FP32, max_steps=128)
    srv = hm.Server(ctx, precision=hm.FP32, max_steps=128, hbm_budget_bytes=1 << 30)
    pool = srv.stats()["pool_bytes"]
    srv.close()
    per_req = 256 + 512 * max(math.ceil(q["n_paths"] / 1024) for q in reqs)
    budget = (1 << 30) - pool + 3 * per_req + 4096
    srv = hm.Server(ctx, precision=hm.FP32, max_steps=128, hbm_budget_bytes=budget)
    try:
        assert srv.stats()["pool_bytes"] < 4 * per_req + 4096
        tickets = [srv.submit(**q) for q in reqs]
        peak_queue = max(srv.stats()["queued"] for _ in range(3))
        small = [srv.wait(t, 120_000) for t in tickets]
        stats = srv.stats()
    finally:
        srv.close()
    assert stats["completed"] == 12 and stats["admitted"] == 12
    assert peak_queue >= 1
    for a, b in zip(big, small):
        assert a["price"] == b["price"]


def test_poll_and_errors(hm, ctx):
    srv = hm.Server(ctx, precision=hm.FP32, max_steps=64)
    try:
        q = requests(1)[0]
        q["n_steps"] = 60
        t = srv.submit(**q)
        r = None
        deadline = time.time() + 60
        while r is None and time.time() < deadline:
            r = srv.poll(t)
        assert r is not None and r["n_paths"] == q["n_paths"]
        with pytest.raises(hm.HestonError) as e:
            srv.poll(t)  # released after the first successful poll
        assert e.value.status == -6
        with pytest.raises(hm.HestonError):
            srv.submit(**dict(q, n_steps=65))  # above max_steps
        with pytest.raises(hm.HestonError):
            srv.submit(**dict(q, want=0))
    finally:
        srv.close()


def test_served_qe_matches_batch(hm, ctx):
    """A server running Andersen's QE scheme: served requests (price and
    adjoint modes, FP32 and FP64) equal the batch API's results up to the
    order in which the FP64 unit records are added (the batch API's QE
    results are checked against the oracle in tests/test_gpu_batch.py)."""
    for prec in (hm.FP32, hm.FP64):
        for want in (1, 2):
            reqs = requests(8, want=want, seed=31)
            res, _ = serve(hm, ctx, reqs, precision=prec, scheme=hm.QE)
            bat, _ = ctx.price_batch(reqs, hm.Options(precision=prec, scheme=hm.QE,
                                                      greeks=hm.GREEKS_PATHWISE))
            for q, r, b in zip(reqs, res, bat):
                assert r["n_paths"] == q["n_paths"]
                for k in ("price", "pw_delta", "pw_rho"):
                    assert r[k][0] == pytest.approx(b[k][0], rel=1e-12, abs=1e-13), (prec, want, k)
                for k in range(7 if want == 2 else 0):
                    assert r["adj"][k][0] == pytest.approx(b["adj"][k][0], rel=1e-12, abs=1e-13)
