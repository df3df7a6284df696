"""CPU oracle for the Heston / Milstein Monte-Carlo path -- TEST INFRASTRUCTURE.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may import
this package.  The product library never calls it and shares no code with it.

Contents
--------
- ``heston_oracle.c`` (built to ``liboracle.so`` with gcc): Philox4x32-10, the
  Box-Muller normals, one Milstein path at a time in FP64 with its payoff and
  pathwise estimators, forward-mode derivatives of the payoff, and Andersen's
  quadratic-exponential (QE) path.
- this module: ctypes marshalling, plus the estimators built on top of the
  per-path records -- means and standard errors (two-pass), central
  bump-and-revalue Greeks on common random numbers by full re-simulation of
  every bumped scenario, and quasi-Monte-Carlo replicate estimates.
- ``analytic``: Heston characteristic-function prices and Greeks, Black-Scholes.
- ``sobol``: Sobol points (Gray-code order, digital shifts) and the Brownian
  bridge, giving quasi-random normals for the same path simulator.
- ``bk``: Broadie-Kaya exact simulation.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass, astuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "heston_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

EURO_CALL, EURO_PUT, ASIAN_CALL, ASIAN_PUT, GEO_ASIAN_CALL, GEO_ASIAN_PUT = 0, 1, 2, 3, 4, 5
(FULL_TRUNC, ABSORB, QE, EULER_FULL_TRUNC, EULER_ABSORB, PARTIAL_TRUNC,
 REFLECT) = 0, 1, 2, 3, 4, 5, 6
REC_FIELDS = ("S_T", "V_T", "Sbar", "pay", "pw_delta", "pw_rho")
TAN_FIELDS = ("pay", "d_S0", "d_v0", "d_r", "d_kappa", "d_theta", "d_sigma", "d_rho",
              "max_dsqrt")
PARAM_NAMES = ("S0", "K", "r", "T", "v0", "kappa", "theta", "sigma", "rho")


@dataclass(frozen=True)
class Params:
    S0: float
    K: float
    r: float
    T: float
    v0: float
    kappa: float
    theta: float
    sigma: float
    rho: float

    def replace(self, **kw) -> "Params":
        d = dict(zip(PARAM_NAMES, astuple(self)))
        d.update(kw)
        return Params(**d)


class _CParams(ctypes.Structure):
    _fields_ = [(n, ctypes.c_double) for n in PARAM_NAMES]


def build(force: bool = False) -> str:
    """Compile liboracle.so with gcc (plain -O2, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-fPIC", "-shared",
                               "-Wall", "-Wextra", "-o", tmp, _SRC, "-lm", "-lpthread"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB)
        P = ctypes.POINTER
        u32p, dp = P(ctypes.c_uint32), P(ctypes.c_double)
        sig = [P(_CParams), ctypes.c_int, ctypes.c_uint32, u32p, ctypes.c_uint32, ctypes.c_int,
               ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64, dp, dp, ctypes.c_int, dp]
        for name in ("or_simulate", "or_tangent"):
            f = getattr(L, name)
            f.argtypes = sig
            f.restype = ctypes.c_int
        L.or_philox_block.argtypes = [u32p, u32p, ctypes.c_uint64, u32p]
        L.or_philox_block.restype = None
        L.or_normals_block.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64,
                                       ctypes.c_uint32, dp, dp]
        L.or_normals_block.restype = None
        L.or_uniform.argtypes = [ctypes.c_uint32]
        L.or_uniform.restype = ctypes.c_double
        L.or_qe_draws.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint32, dp, dp, dp]
        L.or_qe_draws.restype = None
        L.or_qe_draws_block.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64,
                                        ctypes.c_uint32, dp, dp, dp]
        L.or_qe_draws_block.restype = None
        _lib = L
    return _lib


def _ptr(a, ctype):
    return a.ctypes.data_as(ctypes.POINTER(ctype)) if a is not None else None


def philox(ctr, key) -> np.ndarray:
    """Philox4x32-10 words for arrays ctr [n,4] and key [n,2] (uint32)."""
    ctr = np.ascontiguousarray(np.atleast_2d(ctr), dtype=np.uint32)
    key = np.ascontiguousarray(np.atleast_2d(key), dtype=np.uint32)
    n = ctr.shape[0]
    out = np.empty((n, 4), dtype=np.uint32)
    lib().or_philox_block(_ptr(ctr, ctypes.c_uint32), _ptr(key, ctypes.c_uint32), n,
                          _ptr(out, ctypes.c_uint32))
    return out


def normals(seed: int, first: int, n_paths: int, n_steps: int):
    """The Philox/Box-Muller normals (Za, Zb), each [n_paths, n_steps]."""
    za = np.empty((n_paths, n_steps))
    zb = np.empty((n_paths, n_steps))
    lib().or_normals_block(seed, first, n_paths, n_steps, _ptr(za, ctypes.c_double),
                           _ptr(zb, ctypes.c_double))
    return za, zb


def _fix_array(fixings):
    if fixings is None:
        return None, 0
    f = np.ascontiguousarray(fixings, dtype=np.uint32)
    return f, int(f.size)


def simulate(p: Params, opt_type: int, n_steps: int, seed: int = 0, first: int = 0,
             n_paths: int = 1, mode: int = FULL_TRUNC, fixings=None, za=None, zb=None,
             threads: int = 1) -> np.ndarray:
    """Per-path records [n_paths, 6] = (S_T, V_T, Sbar, pay, pw_delta, pw_rho)."""
    if mode == QE:
        return simulate_qe(p, opt_type, n_steps, seed, first, n_paths, fixings, threads)[0]
    return _run("or_simulate", len(REC_FIELDS), p, opt_type, n_steps, seed, first, n_paths, mode,
                fixings, za, zb, threads)


def simulate_qe(p: Params, opt_type: int, n_steps: int, seed: int = 0, first: int = 0,
                n_paths: int = 1, fixings=None, threads: int = 1):
    """Andersen's QE scheme: (records [n_paths, 6] as simulate, margin [n_paths],
    amp [n_paths]).  margin is the path's smallest distance from taking the other
    branch at a step: |psi - 3/2| / (3/2), and |Uv - p| where the exponential branch
    is taken.  amp >= 1 is the path's amplification of relative variance errors:
    max over j of max_{i<=j} V_i |dV_j/dV_i| / max(V_j, v0, theta)."""
    n = len(REC_FIELDS)
    out = _run("or_simulate", n + 2, p, opt_type, n_steps, seed, first, n_paths, QE,
               fixings, None, None, threads)
    return out[:, :n], out[:, n], out[:, n + 1]


def qe_draws(seed: int, path: int, step: int):
    """The QE scheme's random inputs (Zs, Zv, Uv) of one step of one path."""
    zs, zv, uv = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    lib().or_qe_draws(seed & (2**64 - 1), path, step, ctypes.byref(zs), ctypes.byref(zv),
                      ctypes.byref(uv))
    return zs.value, zv.value, uv.value


def qe_draws_block(seed: int, first: int, n_paths: int, n_steps: int):
    """The QE scheme's random inputs (Zs, Zv, Uv), each [n_paths, n_steps]."""
    zs, zv, uv = (np.empty((n_paths, n_steps)) for _ in range(3))
    lib().or_qe_draws_block(seed & (2**64 - 1), first, n_paths, n_steps, _ptr(zs, ctypes.c_double),
                            _ptr(zv, ctypes.c_double), _ptr(uv, ctypes.c_double))
    return zs, zv, uv


def tangent(p: Params, opt_type: int, n_steps: int, seed: int = 0, first: int = 0,
            n_paths: int = 1, mode: int = FULL_TRUNC, fixings=None, za=None, zb=None,
            threads: int = 1) -> np.ndarray:
    """Per-path [n_paths, 9] = (pay, d/dS0, d/dv0, d/dr, d/dkappa, d/dtheta, d/dsigma, d/drho,
    c), with c the largest factor d sqrt(V+ dt)/dV+ = sqrt(dt / V+_j) / 2 on the path
    (Milstein modes), or its smallest branch margin (QE: mode=QE, Philox inputs
    only; the branch decisions are held fixed, so a bump smaller than the
    margin does not move a branch)."""
    return _run("or_tangent", len(TAN_FIELDS), p, opt_type, n_steps, seed, first, n_paths, mode,
                fixings, za, zb, threads)


def _run(fn, width, p, opt_type, n_steps, seed, first, n_paths, mode, fixings, za, zb, threads):
    fix, nf = _fix_array(fixings)
    if za is not None:
        za = np.ascontiguousarray(za, dtype=np.float64)
        zb = np.ascontiguousarray(zb, dtype=np.float64)
        assert za.shape == (n_paths, n_steps) and zb.shape == za.shape
    out = np.empty((n_paths, width))
    cp = _CParams(*astuple(p))
    rc = getattr(lib(), fn)(ctypes.byref(cp), opt_type, n_steps, _ptr(fix, ctypes.c_uint32), nf,
                            mode, seed & (2**64 - 1), first, n_paths, _ptr(za, ctypes.c_double),
                            _ptr(zb, ctypes.c_double), threads, _ptr(out, ctypes.c_double))
    if rc != 0:
        raise ValueError(f"{fn}: invalid argument")
    return out


# --------------------------------------------------------------------------
# Estimators on top of the per-path records.

def mean_se(y: np.ndarray):
    """Sample mean and its standard error, two-pass: sqrt(sum (y-mean)^2 / (n(n-1)))."""
    y = np.asarray(y, dtype=np.float64)
    n = y.shape[0]
    m = y.sum(axis=0) / n
    ss = ((y - m) ** 2).sum(axis=0)
    return m, np.sqrt(ss / (n * (n - 1)))


@dataclass(frozen=True)
class Bumps:
    """Central bump sizes: relative for S0 and v0, absolute for r and T."""
    S0_rel: float = 0.01
    v0_rel: float = 0.01
    r_abs: float = 1e-4
    T_abs: float = 1.0 / 365.0


SCENARIOS = ("base", "S0+", "S0-", "v0+", "v0-", "r+", "r-", "T+", "T-")


def scenario_params(p: Params, b: Bumps):
    hS, hv = b.S0_rel * p.S0, b.v0_rel * p.v0
    return {
        "base": p,
        "S0+": p.replace(S0=p.S0 + hS), "S0-": p.replace(S0=p.S0 - hS),
        "v0+": p.replace(v0=p.v0 + hv), "v0-": p.replace(v0=p.v0 - hv),
        "r+": p.replace(r=p.r + b.r_abs), "r-": p.replace(r=p.r - b.r_abs),
        "T+": p.replace(T=p.T + b.T_abs), "T-": p.replace(T=p.T - b.T_abs),
    }


def scenario_payoffs(p: Params, opt_type: int, n_steps: int, seed: int, n_paths: int,
                     first: int = 0, mode: int = FULL_TRUNC, fixings=None, bumps: Bumps = Bumps(),
                     za=None, zb=None, threads: int = 1):
    """Per-path discounted payoffs of all 9 scenarios on common random numbers.

    Every scenario is a complete re-simulation with the bumped parameter; the
    step count N and the fixing step indices stay fixed, so a T bump rescales
    dt and the fixing times."""
    out = {}
    base_rec = None
    for name, q in scenario_params(p, bumps).items():
        rec = simulate(q, opt_type, n_steps, seed, first, n_paths, mode, fixings, za, zb, threads)
        out[name] = rec[:, 3]
        if name == "base":
            base_rec = rec
    return out, base_rec


def greek_samples(pay: dict, p: Params, bumps: Bumps = Bumps()):
    """Per-path central-difference Greek samples (their means are the Greeks)."""
    hS, hv = bumps.S0_rel * p.S0, bumps.v0_rel * p.v0
    return {
        "price": pay["base"],
        "delta": (pay["S0+"] - pay["S0-"]) / (2 * hS),
        "gamma": (pay["S0+"] - 2 * pay["base"] + pay["S0-"]) / (hS * hS),
        "vega": (pay["v0+"] - pay["v0-"]) / (2 * hv),
        "rho": (pay["r+"] - pay["r-"]) / (2 * bumps.r_abs),
        "theta": -(pay["T+"] - pay["T-"]) / (2 * bumps.T_abs),
    }


def price_greeks(p: Params, opt_type: int, n_paths: int, n_steps: int, seed: int,
                 mode: int = FULL_TRUNC, fixings=None, bumps: Bumps | None = Bumps(),
                 threads: int = 1, first: int = 0):
    """Price, pathwise Delta/Rho and (optionally) the five bump Greeks.

    Returns {name: (value, std_err)} over the paths first .. first+n_paths-1."""
    if bumps is not None:
        pay, rec = scenario_payoffs(p, opt_type, n_steps, seed, n_paths, first, mode, fixings,
                                    bumps, threads=threads)
        samples = greek_samples(pay, p, bumps)
    else:
        rec = simulate(p, opt_type, n_steps, seed, first, n_paths, mode, fixings, threads=threads)
        samples = {"price": rec[:, 3]}
    samples["pw_delta"] = rec[:, 4]
    samples["pw_rho"] = rec[:, 5]
    return {k: tuple(float(v) for v in mean_se(y)) for k, y in samples.items()}


# --------------------------------------------------------------------------
# Geometric-average control variate for the arithmetic Asian (the paper notes
# that the average may be geometric; using the geometric payoff, whose price
# has a semi-analytic form, as a control follows Kemna and Vorst, 1990).

def control_variate(a: np.ndarray, g: np.ndarray, mu: float):
    """Control-variate estimate from per-path arithmetic payoffs a and geometric
    payoffs g on the same paths, with E[g] = mu known.

    beta = Cov(a, g) / Var(g) (sample moments, n - 1 denominators; 0 when g is
    constant); estimate = mean(a) - beta (mean(g) - mu); its standard error is
    sqrt((Var(a) - beta Cov(a, g)) / n), the residual variance of a - beta g.
    Returns (estimate, std_err, beta)."""
    a = np.asarray(a, dtype=np.float64)
    g = np.asarray(g, dtype=np.float64)
    n = a.shape[0]
    ma, mg = a.sum() / n, g.sum() / n
    va = ((a - ma) ** 2).sum() / (n - 1)
    vg = ((g - mg) ** 2).sum() / (n - 1)
    cov = ((a - ma) * (g - mg)).sum() / (n - 1)
    beta = cov / vg if vg > 0 else 0.0
    res = max(va - beta * cov, 0.0)
    return ma - beta * (mg - mu), math.sqrt(res / n), beta


def control_variate_reps(a: np.ndarray, g: np.ndarray, mu: float, R: int):
    """Replicated (quasi-random) form: the paths are R equal replicates in order;
    beta comes from all paths as in control_variate, each replicate gives
    mean(a_r) - beta (mean(g_r) - mu), and the estimate and its standard error
    are the mean of those R values and their std (ddof 1) / sqrt(R)."""
    _, _, beta = control_variate(a, g, mu)
    a = np.asarray(a, dtype=np.float64).reshape(R, -1)
    g = np.asarray(g, dtype=np.float64).reshape(R, -1)
    e = a.mean(axis=1) - beta * (g.mean(axis=1) - mu)
    m = e.sum() / R
    return m, math.sqrt(((e - m) ** 2).sum() / (R - 1) / R), beta


def geometric_control_mean(p: Params, opt_type: int, n_steps: int, fixings=None) -> float:
    """E of the discounted geometric payoff matching an arithmetic Asian type
    (call for ASIAN_CALL, put for ASIAN_PUT) on the same fixing dates."""
    from . import analytic
    steps = np.arange(1, n_steps + 1) if fixings is None else np.asarray(fixings)
    t = steps / n_steps * p.T
    if opt_type == ASIAN_CALL:
        return analytic.geometric_asian_call(p, t)
    if opt_type == ASIAN_PUT:
        return analytic.geometric_asian_put(p, t)
    raise ValueError("the geometric control applies to arithmetic Asian types")


def cv_price(p: Params, opt_type: int, n_paths: int, n_steps: int, seed: int,
             mode: int = FULL_TRUNC, fixings=None, threads: int = 1, first: int = 0):
    """Arithmetic-Asian price with the geometric control on the same paths.
    Returns (estimate, std_err, beta, mu, a, g)."""
    geo = GEO_ASIAN_CALL if opt_type == ASIAN_CALL else GEO_ASIAN_PUT
    mu = geometric_control_mean(p, opt_type, n_steps, fixings)
    a = simulate(p, opt_type, n_steps, seed, first, n_paths, mode, fixings, threads=threads)[:, 3]
    g = simulate(p, geo, n_steps, seed, first, n_paths, mode, fixings, threads=threads)[:, 3]
    est, se, beta = control_variate(a, g, mu)
    return est, se, beta, mu, a, g
