"""Pins of the CPU oracle against facts outside itself (no GPU needed).

Each test names the passage of the paper it checks and the independent fact
it uses: a library run here (rocRAND's Philox engine, scipy/torch Sobol,
scipy quadrature), a closed form, an exact identity, brute force, or a value
printed in the paper (tests/golden/paper_values.json).
"""
import json
import math
import os
import shutil
import subprocess

import numpy as np
import pytest
from scipy import stats

import oracle
from oracle import analytic, sobol
from workloads import BASE, PAPER, paper_fixing_steps

HERE = os.path.dirname(os.path.abspath(__file__))
GOLD = json.load(open(os.path.join(HERE, "golden", "paper_values.json")))
PB = oracle.Params(**BASE)
PP = oracle.Params(**PAPER)
EC, EP, AC, AP = oracle.EURO_CALL, oracle.EURO_PUT, oracle.ASIAN_CALL, oracle.ASIAN_PUT


# --------------------------------------------------------------------------
# Philox4x32-10 against rocRAND's header-only engine, run on the host.

@pytest.fixture(scope="session")
def rocrand_ref(tmp_path_factory):
    if shutil.which("g++") is None or not os.path.exists("/opt/rocm/include/rocrand"):
        pytest.skip("g++ or rocRAND headers not available")
    exe = str(tmp_path_factory.mktemp("pins") / "rocrand_philox_ref")
    subprocess.check_call(["g++", "-O1", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
                           os.path.join(HERE, "pins", "rocrand_philox_ref.cpp"), "-o", exe])
    return exe


def test_philox_matches_rocrand(rocrand_ref):
    g = np.random.default_rng(1)
    key = g.integers(0, 2**32, (300, 2), dtype=np.uint64).astype(np.uint32)
    ctr = g.integers(0, 2**32, (300, 4), dtype=np.uint64).astype(np.uint32)
    key[:4] = [[0, 0], [0xFFFFFFFF, 0xFFFFFFFF], [42, 0], [7, 1]]
    ctr[:4] = [[0, 0, 0, 0], [0xFFFFFFFF] * 4, [0, 5, 0, 0], [1, 2, 3, 4]]
    lines = "\n".join(" ".join(str(int(v)) for v in (*k, *c)) for k, c in zip(key, ctr))
    out = subprocess.run([rocrand_ref], input=lines, capture_output=True, text=True, check=True)
    ref = np.array([[int(v) for v in ln.split()] for ln in out.stdout.strip().splitlines()],
                   dtype=np.uint64)
    mine = oracle.philox(ctr, key).astype(np.uint64)
    assert np.array_equal(mine, ref)


def test_uniform_mapping_is_exact_in_single_precision():
    L = oracle.lib()
    for w, expect in [(0, 2.0**-24), (0xFFFFFFFF, 1.0 - 2.0**-24), (1 << 9, 1.5 * 2.0**-23),
                      (0x80000000, 0.5 + 2.0**-24)]:
        u = L.or_uniform(w)
        assert u == expect
        assert float(np.float32(u)) == u
    ws = np.random.default_rng(2).integers(0, 2**32, 10000, dtype=np.uint64)
    us = np.array([L.or_uniform(int(w)) for w in ws[:2000]])
    assert np.all((us > 0) & (us < 1))
    assert np.array_equal(us.astype(np.float32).astype(np.float64), us)


def test_box_muller_geometry_and_stream_layout():
    """Za^2+Zb^2 = -2 ln ua and atan2(Zb, Za) = 2 pi ub for the words of the
    stated counter layout; even/odd steps share one Philox block."""
    seed, first, n, N = 0x123456789ABC, 1000, 64, 6
    za, zb = oracle.normals(seed, first, n, N)
    for p in range(0, n, 9):
        for j in range(N):
            path = first + p
            w = oracle.philox([[j >> 1, path & 0xFFFFFFFF, path >> 32, 0]],
                              [[seed & 0xFFFFFFFF, seed >> 32]])[0]
            wa, wb = (w[2], w[3]) if j & 1 else (w[0], w[1])
            ua = ((int(wa) >> 9) + 0.5) / 2**23
            ub = ((int(wb) >> 9) + 0.5) / 2**23
            assert za[p, j] ** 2 + zb[p, j] ** 2 == pytest.approx(-2 * math.log(ua), rel=1e-13)
            ang = math.atan2(zb[p, j], za[p, j]) % (2 * math.pi)
            assert ang == pytest.approx(2 * math.pi * ub, abs=1e-12)


def test_normals_are_standard_and_independent():
    za, zb = oracle.normals(42, 0, 4096, 64)
    z = np.concatenate([za.ravel(), zb.ravel()])
    assert stats.kstest(z, "norm").pvalue > 1e-3
    assert abs(z.mean()) < 4 / math.sqrt(z.size)
    assert abs(z.var() - 1) < 6 * math.sqrt(2 / z.size)
    n = za.size
    for a, b in [(za.ravel(), zb.ravel()), (za[:, :-1].ravel(), za[:, 1:].ravel()),
                 (za[:-1].ravel(), za[1:].ravel())]:
        assert abs(np.corrcoef(a, b)[0, 1]) < 5 / math.sqrt(n)


# --------------------------------------------------------------------------
# Milstein scheme (paper: algorithm "Milstein approximation under Heston model").

def test_one_step_price_closed_form():
    """N=1: ln(S_1/S0) = (r - v0/2) T + sqrt(v0 T) Za, for any kappa, theta, sigma, rho."""
    p = PB.replace(kappa=3.0, theta=0.09, sigma=0.9, rho=0.4)
    rec = oracle.simulate(p, EC, 1, seed=7, n_paths=500)
    za, _ = oracle.normals(7, 0, 500, 1)
    expect = p.S0 * np.exp((p.r - 0.5 * p.v0) * p.T + np.sqrt(p.v0 * p.T) * za[:, 0])
    assert np.allclose(rec[:, 0], expect, rtol=1e-14, atol=0)


@pytest.mark.parametrize("rho", [-0.7, 0.0, 0.95])
def test_one_step_variance_completed_square(rho):
    """One Milstein variance step is the completed square
    (sqrt(v0) + sigma sqrt(dt) Z2 / 2)^2 + (kappa(theta - v0) - sigma^2/4) dt,
    with Z2 = rho Za + sqrt(1-rho^2) Zb."""
    p = PB.replace(rho=rho, sigma=0.7, v0=0.05)
    rec = oracle.simulate(p, EC, 1, seed=9, n_paths=400)
    za, zb = oracle.normals(9, 0, 400, 1)
    z2 = rho * za[:, 0] + math.sqrt(1 - rho * rho) * zb[:, 0]
    dt = p.T
    expect = (math.sqrt(p.v0) + 0.5 * p.sigma * math.sqrt(dt) * z2) ** 2 \
        + (p.kappa * (p.theta - p.v0) - 0.25 * p.sigma ** 2) * dt
    assert np.allclose(rec[:, 1], expect, rtol=1e-12, atol=1e-15)


def test_sigma_zero_closed_form_path():
    """sigma = 0: V_j = theta + (v0 - theta)(1 - kappa dt)^j is deterministic and
    S_T = S0 exp(rT - sum V_j dt / 2 + sum sqrt(V_j dt) Za_j)."""
    N = 37
    p = PB.replace(sigma=0.0, v0=0.09, theta=0.02, kappa=3.0)
    dt = p.T / N
    rec = oracle.simulate(p, EC, N, seed=11, n_paths=300)
    za, _ = oracle.normals(11, 0, 300, N)
    V = p.theta + (p.v0 - p.theta) * (1 - p.kappa * dt) ** np.arange(N)
    lnS = p.r * p.T - 0.5 * V.sum() * dt + (np.sqrt(V * dt)[None, :] * za).sum(axis=1)
    assert np.allclose(rec[:, 0], p.S0 * np.exp(lnS), rtol=1e-12, atol=0)
    assert np.allclose(rec[:, 1], p.theta + (p.v0 - p.theta) * (1 - p.kappa * dt) ** N, rtol=1e-12)


def test_sigma_zero_black_scholes_limit():
    """sigma = 0, v0 = theta: constant variance, the log-Euler step is exact for
    geometric Brownian motion, so the price is Black-Scholes at vol sqrt(theta)."""
    p = PB.replace(sigma=0.0, v0=0.04, theta=0.04)
    r = oracle.price_greeks(p, EC, 1 << 17, 16, seed=3, bumps=None, threads=8)
    bs = analytic.bs_call_greeks(p.S0, p.K, p.r, p.T, 0.2)
    for k in ("price", "pw_delta", "pw_rho"):
        key = {"price": "price", "pw_delta": "delta", "pw_rho": "rho"}[k]
        assert abs(r[k][0] - bs[key]) < 3.5 * r[k][1]


@pytest.mark.parametrize("mode", [oracle.FULL_TRUNC, oracle.ABSORB])
def test_martingale(mode):
    """exp(-rT) E[S_T] = S0: the discrete log-price step is an exact martingale given V."""
    p = PP  # Feller condition violated: 2 kappa theta < sigma^2
    rec = oracle.simulate(p, EC, 64, seed=5, n_paths=1 << 16, mode=mode, threads=8)
    m, se = oracle.mean_se(math.exp(-p.r * p.T) * rec[:, 0])
    assert abs(m - p.S0) < 3.5 * se


def test_asian_average_mean():
    N = 50
    fix = np.array([5, 17, 30, 50])
    rec = oracle.simulate(PB, AC, N, seed=5, n_paths=1 << 15, fixings=fix, threads=8)
    t = fix * PB.T / N
    m, se = oracle.mean_se(rec[:, 2])
    assert abs(m - PB.S0 * np.exp(PB.r * t).mean()) < 3.5 * se


@pytest.mark.parametrize("asian", [False, True])
def test_put_call_identity_per_path(asian):
    c, pt = (AC, AP) if asian else (EC, EP)
    rc = oracle.simulate(PB, c, 30, seed=1, n_paths=2000)
    rp = oracle.simulate(PB, pt, 30, seed=1, n_paths=2000)
    D = math.exp(-PB.r * PB.T)
    X = rc[:, 2]
    assert np.allclose(rc[:, 3] - rp[:, 3], D * (X - PB.K), rtol=0, atol=1e-12)
    assert np.allclose(rc[:, 4] - rp[:, 4], D * X / PB.S0, rtol=0, atol=1e-14)


def test_absorption_keeps_variance_nonnegative():
    rf = oracle.simulate(PP, EC, 32, seed=2, n_paths=4000, mode=oracle.FULL_TRUNC)
    ra = oracle.simulate(PP, EC, 32, seed=2, n_paths=4000, mode=oracle.ABSORB)
    assert ra[:, 1].min() >= 0.0
    assert rf[:, 1].min() < 0.0  # Feller violated: the unclamped variance goes negative


def test_asian_single_fixing_reduces_to_european():
    """With one fixing at T the Asian payoff and estimators equal the European
    ones (the Asian Rho estimator as derived reduces to e^{-rT} K T 1{S_T>K})."""
    N = 20
    e = oracle.simulate(PB, EC, N, seed=4, n_paths=3000)
    a = oracle.simulate(PB, AC, N, seed=4, n_paths=3000, fixings=[N])
    assert np.allclose(e[:, 3:], a[:, 3:], rtol=1e-13, atol=1e-12)


@pytest.mark.parametrize("opt", [EC, EP, AC, AP])
def test_pathwise_estimators_are_exact_derivatives(opt):
    """Pathwise Delta and Rho equal central differences of the same path's
    discounted payoff on common random numbers (S0 and r bumps re-simulate)."""
    N, n = 24, 3000
    rec = oracle.simulate(PB, opt, N, seed=8, n_paths=n)
    hS, hr = 1e-5 * PB.S0, 1e-7
    up = oracle.simulate(PB.replace(S0=PB.S0 + hS), opt, N, seed=8, n_paths=n)[:, 3]
    dn = oracle.simulate(PB.replace(S0=PB.S0 - hS), opt, N, seed=8, n_paths=n)[:, 3]
    fd_delta = (up - dn) / (2 * hS)
    up = oracle.simulate(PB.replace(r=PB.r + hr), opt, N, seed=8, n_paths=n)[:, 3]
    dn = oracle.simulate(PB.replace(r=PB.r - hr), opt, N, seed=8, n_paths=n)[:, 3]
    fd_rho = (up - dn) / (2 * hr)
    smooth = np.abs(rec[:, 2] - PB.K) > 1e-3 * PB.K
    assert smooth.mean() > 0.98
    assert np.allclose(rec[smooth, 4], fd_delta[smooth], rtol=1e-6, atol=1e-8)
    assert np.allclose(rec[smooth, 5], fd_rho[smooth], rtol=1e-6, atol=1e-5)


@pytest.mark.parametrize("opt,mode", [(EC, oracle.FULL_TRUNC), (AC, oracle.FULL_TRUNC),
                                      (EP, oracle.ABSORB), (AP, oracle.FULL_TRUNC)])
def test_tangent_matches_finite_differences(opt, mode):
    """Forward-mode derivatives vs central differences per path, all seven
    parameters; paths whose payoff is not smooth between the bumps (kink or a
    truncation switch) are recognised by disagreement of two step sizes."""
    N, n = 40, 1500
    p = PB.replace(sigma=0.5)
    tan = oracle.tangent(p, opt, N, seed=12, n_paths=n, mode=mode)
    base = oracle.simulate(p, opt, N, seed=12, n_paths=n, mode=mode)
    assert np.allclose(tan[:, 0], base[:, 3], rtol=1e-13, atol=1e-13)
    names = ["S0", "v0", "r", "kappa", "theta", "sigma", "rho"]
    for k, name in enumerate(names):
        x0 = getattr(p, name)
        fds = []
        for h in (1e-5 * max(abs(x0), 0.1), 0.5e-5 * max(abs(x0), 0.1)):
            up = oracle.simulate(p.replace(**{name: x0 + h}), opt, N, seed=12, n_paths=n,
                                 mode=mode)[:, 3]
            dn = oracle.simulate(p.replace(**{name: x0 - h}), opt, N, seed=12, n_paths=n,
                                 mode=mode)[:, 3]
            fds.append((up - dn) / (2 * h))
        scale = np.maximum(np.abs(fds[1]), 1e-3 * np.abs(fds[1]).max() + 1e-12)
        smooth = np.abs(fds[0] - fds[1]) < 1e-6 * scale
        assert smooth.mean() > 0.9, name
        err = np.abs(tan[smooth, 1 + k] - fds[1][smooth]) / scale[smooth]
        assert err.max() < 1e-5, (name, err.max())


def test_tangent_S0_and_r_equal_pathwise_estimators():
    for opt in (EC, EP, AC, AP):
        tan = oracle.tangent(PB, opt, 30, seed=13, n_paths=2000)
        rec = oracle.simulate(PB, opt, 30, seed=13, n_paths=2000)
        assert np.allclose(tan[:, 1], rec[:, 4], rtol=1e-12, atol=1e-14)
        assert np.allclose(tan[:, 3], rec[:, 5], rtol=1e-11, atol=1e-11)


# --------------------------------------------------------------------------
# Analytic references.

def test_characteristic_function_reproduces_paper_values():
    g = GOLD["european_call_analytic"]
    gg = GOLD["european_greeks_analytic"]
    P1, P2 = analytic.probabilities(PP)
    price = analytic.heston_call(PP)
    rho = PP.K * PP.T * math.exp(-PP.r * PP.T) * P2
    assert round(price, 4) == g["value"]
    assert round(P1, 4) == gg["delta"]
    assert round(rho, 4) == gg["rho"]


@pytest.mark.parametrize("p", [PB, PP, PB.replace(rho=0.0), PB.replace(T=0.1, K=90.0),
                               PP.replace(rho=-0.9, K=120.0, T=3.0)])
def test_gil_pelaez_agrees_with_lewis(p):
    assert analytic.heston_call(p) == pytest.approx(analytic.heston_call_lewis(p), abs=1e-9)


def test_characteristic_function_black_scholes_limit():
    p = PB.replace(sigma=1e-5, v0=0.04, theta=0.04)
    assert analytic.heston_call(p) == pytest.approx(analytic.bs_call(100, 100, 0.05, 1, 0.2),
                                                    abs=1e-5)


def test_closed_form_greeks_match_differences_of_price():
    h = 1e-3
    fd = (analytic.heston_call(PB.replace(S0=PB.S0 + h)) -
          analytic.heston_call(PB.replace(S0=PB.S0 - h))) / (2 * h)
    g = analytic.heston_call_greeks(PB)
    assert g["delta"] == pytest.approx(fd, abs=1e-7)
    fd = (analytic.heston_call(PB.replace(r=PB.r + 1e-5)) -
          analytic.heston_call(PB.replace(r=PB.r - 1e-5))) / 2e-5
    assert g["rho"] == pytest.approx(fd, abs=1e-5)


# --------------------------------------------------------------------------
# Statistical agreement with the analytic values and the paper's tables.

@pytest.mark.slow
def test_milstein_european_matches_analytic():
    g = analytic.heston_call_greeks(PB)
    r = oracle.price_greeks(PB, EC, 1 << 17, 100, seed=42, threads=8)
    bias = {"price": 0.01, "delta": 5e-4, "gamma": 2e-4, "vega": 0.2, "rho": 0.1, "theta": 0.05,
            "pw_delta": 5e-4, "pw_rho": 0.1}
    for k, (v, se) in r.items():
        ref = g[{"pw_delta": "delta", "pw_rho": "rho"}.get(k, k)]
        assert abs(v - ref) < 4 * se + bias[k], (k, v, se, ref)


@pytest.mark.slow
@pytest.mark.parametrize("asian", [False, True])
def test_milstein_reproduces_paper_tables(asian):
    """Paper parameters, 32 000 paths: the CPU Milstein prices of the paper's
    step tables (30-run mean and std) against one run of ours."""
    key = "milstein_asian_cpu_32000_paths" if asian else "milstein_european_cpu_32000_paths"
    tab = GOLD[key]
    for N, val, std in zip(tab["steps"], tab["value"], tab["std"]):
        fix = paper_fixing_steps(N) if asian else None
        rec = oracle.simulate(PP, AC if asian else EC, N, seed=N, n_paths=32000, fixings=fix,
                              mode=oracle.ABSORB, threads=8)
        m, se = oracle.mean_se(rec[:, 3])
        assert abs(m - val) < 4 * math.hypot(se, std), (N, m, se, val, std)


@pytest.mark.parametrize("asian", [False, True])
def test_milstein_reproduces_paper_path_count_tables(asian):
    """Paper parameters, 128 steps, 4000 to 32 000 paths: the CPU Milstein
    prices of the paper's path-count tables (30-run mean and std)."""
    key = "milstein_asian_paths_128_steps" if asian else "milstein_european_paths_128_steps"
    tab = GOLD[key]
    for n, val, std in zip(tab["paths"], tab["value"], tab["std"]):
        rec = oracle.simulate(PP, AC if asian else EC, 128, seed=2000 + n, n_paths=n,
                              fixings=paper_fixing_steps(128) if asian else None,
                              mode=oracle.ABSORB, threads=8)
        m, se = oracle.mean_se(rec[:, 3])
        assert abs(m - val) < 4 * math.hypot(se, std), (n, m, se, val, std)


@pytest.mark.slow
def test_milstein_asian_matches_paper_exact_simulation():
    g = GOLD["asian_bk_qmc_512"]
    rec = oracle.simulate(PP, AC, 128, seed=17, n_paths=1 << 18, fixings=paper_fixing_steps(128),
                          mode=oracle.ABSORB, threads=8)
    m, se = oracle.mean_se(rec[:, 3])
    assert abs(m - g["value"]) < 3 * math.hypot(se, g["std"])


def test_asian_pathwise_greeks_near_exact_simulation_values():
    """Paper parameters, quarterly fixings, absorption, 128 steps: the pathwise
    Asian Delta and the corrected Asian Rho against the exact-simulation values
    of the paper's Greeks table (0.6733, 38.1664).  Those values carry
    Monte-Carlo error of their own that the paper does not print, so the bar is
    4 SE plus 0.5%; the printed Rho estimator (with its K T factor) gives
    about 3834, and the paper's own GPU Rho 30.3 misses by 20%."""
    g = GOLD["greeks_table"]["asian"]
    rec = oracle.simulate(PP, AC, 128, seed=41, n_paths=1 << 17, fixings=paper_fixing_steps(128),
                          mode=oracle.ABSORB, threads=8)
    for k, ref in ((4, g["ex_delta"]), (5, g["ex_rho"])):
        m, se = oracle.mean_se(rec[:, k])
        assert abs(m - ref) < 4 * se + 0.005 * ref, (k, m, se, ref)


# --------------------------------------------------------------------------
# Quasi-random normals.

def test_sobol_points_match_torch_engine():
    torch = pytest.importorskip("torch")
    for dim, first, n in [(504, 0, 1024), (20, 777, 300), (2, 65530, 12)]:
        e = torch.quasirandom.SobolEngine(dim, scramble=False)
        if first:
            e.fast_forward(first)
        x = e.draw(n, dtype=torch.float64).numpy()
        assert np.array_equal(sobol.points(dim, first, n), np.rint(x * 2**30).astype(np.uint64))


def test_direction_numbers_torch_equal_scipy():
    """The GPU path takes its direction numbers from torch's SobolEngine; they
    are the table scipy's generator uses."""
    torch = pytest.importorskip("torch")
    import scipy.stats._sobol as ss
    v = np.empty((504, 30), dtype=np.uint32)
    ss._initialize_v(v, 504, 30)
    t = torch.quasirandom.SobolEngine(504, scramble=False).sobolstate.numpy()
    assert np.array_equal(t.astype(np.uint64), v.astype(np.uint64))


@pytest.mark.parametrize("N", [1, 2, 3, 7, 16, 252])
def test_bridge_is_an_orthonormal_map(N):
    """The bridge is linear, z -> increments; unit-variance independent
    increments mean its matrix M satisfies M M^T = I."""
    M = sobol.bridge(np.eye(N))
    assert np.allclose(M @ M.T, np.eye(N), atol=1e-12)
    plan = sobol.bridge_plan(N)
    assert sorted(m for m, _, _ in plan) == list(range(1, N + 1))
    if N == 1:
        assert np.allclose(sobol.bridge(np.array([[0.3]])), [[0.3]])


def test_qmc_replicates_price():
    """Quasi-random European price (16 shifted replicates) within 3 SE + bias
    of the analytic value, and a smaller replicate SE than pseudo-random paths."""
    N, R, M = 64, 16, 2048
    za, zb = sobol.normals(N, 0, R * M, R, M, seed=42)
    rec = oracle.simulate(PB, EC, N, n_paths=R * M, za=za, zb=zb, threads=8)
    means = rec[:, 3].reshape(R, M).mean(axis=1)
    q, qse = means.mean(), means.std(ddof=1) / math.sqrt(R)
    ref = analytic.heston_call(PB)
    assert abs(q - ref) < 3 * qse + 0.02
    mc = oracle.simulate(PB, EC, N, seed=42, n_paths=R * M, threads=8)
    assert qse < oracle.mean_se(mc[:, 3])[1]
