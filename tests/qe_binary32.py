"""The QE step evaluated in binary32 on the CPU -- test infrastructure.

The single-precision pricing kernel evaluates Andersen's QE scheme in a
scaled state (y = ln(S/S0)/ln 2 without the drift r t, w = V dt) with binary32
arithmetic.  This module evaluates the same formulas, in the same order and
state, with numpy on the CPU, so the parity tests can tell how far any binary32
evaluation of those formulas lands from the FP64 oracle on a given path.  It
is not the oracle (whose arithmetic it does not share) and not the GPU path
(nothing here is called by the library); it imports only the oracle's Philox
words, the same random inputs both sides consume.

Why it is needed: a QE variance step maps a small variance to a large one
with a large derivative where the vol of vol is high (|dV'/dV| above 10), so a
relative rounding error of the variance at one step reappears multiplied in
every later variance and log-price increment.  Any binary32 evaluation of
such a path differs from the exact one by far more than one rounding; how much
depends on the path.

Two modes:
- round to nearest (``ensemble=0``): one deterministic binary32 evaluation,
  fused multiply-adds where the kernel's compiler contracts them;
- Monte Carlo arithmetic (Parker, 1997, "Monte Carlo Arithmetic: exploiting
  randomness in floating-point arithmetic"): each operation's exact result is
  multiplied by (1 + xi 2^-24 ulps), xi uniform in [-1, 1], before rounding,
  with ``ulps`` 1 for arithmetic and the hardware's measured accuracy for the
  transcendental instructions (log2, exp2, sqrt, reciprocal 1 ulp; sin and cos
  of an angle in revolutions 1.3e-7 absolute).  ``spread`` runs an ensemble of
  such evaluations and returns, per path and record column, the largest
  distance from the oracle: an estimate of how far a binary32 evaluation with
  that rounding behaviour can land on that path.

With ``dtype=np.float64`` and no perturbation the same code is an FP64
evaluation of the kernel's formulation; tests check it against the oracle to
1e-11, which pins this module's formulas to the oracle's arithmetic.

Record columns (as ``heston_dump_paths``): 0 S_T, 1 V_T, 2 the averaged
price (S_T for Europeans), 3 payoff, 4 pathwise Delta, 5 pathwise Rho,
6..13 the payoffs of the bump scenarios S0+, S0-, v0+, v0-, r+, r-, T+, T-
(NaN without bumps).
"""
from __future__ import annotations

import math

import numpy as np

import oracle

LOG2E = 1.4426950408889634074
LN2 = 0.69314718055994530942
QE_TAG = 4
SIN_COS_ABS = 1.3e-7  # measured absolute accuracy of v_sin/v_cos_f32 on 2 pi u


class _Arith:
    """Rounded operations of one evaluation: exact result in binary64, an
    optional relative perturbation, then rounding to the working type."""

    def __init__(self, dtype, rng=None, ulps=1.0):
        self.t = dtype
        self.rng = rng
        self.u = ulps * (2.0 ** -24 if dtype == np.float32 else 2.0 ** -53)

    def r(self, x, ulps=1.0):
        x = np.asarray(x, dtype=np.float64)
        if self.rng is not None:
            x = x * (1.0 + self.rng.uniform(-1.0, 1.0, x.shape) * self.u * ulps)
        return x.astype(self.t)

    def c(self, v):  # a constant rounded once on the host
        return self.t(v)

    def add(self, a, b):
        return self.r(a.astype(np.float64) + b)

    def sub(self, a, b):
        return self.r(a.astype(np.float64) - b)

    def mul(self, a, b):
        return self.r(np.asarray(a, np.float64) * b)

    def fma(self, a, b, c):
        return self.r(np.asarray(a, np.float64) * b + c)

    def sqrt(self, a):
        return self.r(np.sqrt(np.maximum(np.asarray(a, np.float64), 0.0)))

    def rcp(self, a):
        return self.r(1.0 / np.asarray(a, np.float64))

    def log2(self, a):
        return self.r(np.log2(np.asarray(a, np.float64)))

    def exp2(self, a):
        return self.r(np.exp2(np.asarray(a, np.float64)))

    def cos_rev(self, u):  # cos(2 pi u), absolute accuracy of the hardware
        v = np.cos(2.0 * np.pi * np.asarray(u, np.float64))
        if self.rng is not None:
            v = v + self.rng.uniform(-1.0, 1.0, v.shape) * (SIN_COS_ABS if self.t == np.float32 else 0.0)
        return v.astype(self.t)

    def sin_rev(self, u):
        v = np.sin(2.0 * np.pi * np.asarray(u, np.float64))
        if self.rng is not None:
            v = v + self.rng.uniform(-1.0, 1.0, v.shape) * (SIN_COS_ABS if self.t == np.float32 else 0.0)
        return v.astype(self.t)


def _draws(seed, first, n, j):
    """Philox words of the QE block of step j for paths first .. first+n-1."""
    paths = np.arange(first, first + n, dtype=np.uint64)
    ctr = np.stack([np.full(n, j, np.uint32), (paths & 0xFFFFFFFF).astype(np.uint32),
                    (paths >> np.uint64(32)).astype(np.uint32), np.full(n, QE_TAG, np.uint32)], 1)
    key = np.tile(np.array([seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF], np.uint32), (n, 1))
    return oracle.philox(ctr, key)


def _uniform(w):
    """((w >> 9) + 1/2) 2^-23, exact in binary32 and binary64."""
    return ((w >> 9).astype(np.float64) + 0.5) * 2.0 ** -23


class _Grid:
    """QE constants of one time grid, each computed in FP64 and rounded once."""

    def __init__(self, A, p, dt):
        E = math.exp(-p.kappa * dt)
        s2s = p.sigma * p.sigma
        kr = p.kappa * p.rho / p.sigma - 0.5
        self.E = A.c(E)
        self.mth = A.c(p.theta * dt * (1.0 - E))
        self.cs1 = A.c(s2s * dt * E * (1.0 - E) / p.kappa)
        self.cs0 = A.c(p.theta * s2s * dt * dt * (1.0 - E) ** 2 / (2.0 * p.kappa))
        self.k0 = A.c(-p.rho * p.kappa * p.theta * dt / p.sigma * LOG2E)
        self.k1 = A.c((0.5 * dt * kr - p.rho / p.sigma) / dt * LOG2E)
        self.k2 = A.c((0.5 * dt * kr + p.rho / p.sigma) / dt * LOG2E)
        self.k3 = A.c(0.5 * (1.0 - p.rho * p.rho))
        self.k4 = self.k3


def _step(A, g, y, w, z1l, zv, uv):
    """One QE step of one scenario (the kernel's qe_pre + qe_post)."""
    one, two, half = A.c(1.0), A.c(2.0), A.c(0.5)
    m = A.fma(w, g.E, g.mth)
    s2 = A.fma(w, g.cs1, g.cs0)
    rm = A.rcp(m)
    psi = A.mul(A.mul(s2, rm), rm)
    with np.errstate(all="ignore"):
        inv = A.mul(A.mul(A.mul(two, m), m), A.rcp(s2))
        im1 = A.sub(inv, one)
        b2 = A.add(im1, A.sqrt(A.mul(inv, im1)))
        b = A.sqrt(b2)
        a = A.mul(m, A.rcp(A.add(one, b2)))
        bz = A.add(b, zv)
        wq = A.mul(A.mul(a, bz), bz)
        pp1 = A.add(psi, one)
        zero = A.mul(uv, pp1) <= A.sub(psi, one)
        lg = A.mul(A.log2(A.mul(A.mul(half, pp1), A.sub(one, uv))), A.c(LN2))
        we = np.where(zero, A.c(0.0), A.mul(-A.mul(A.mul(half, m), pp1), lg)).astype(A.t)
    wn = np.where(psi <= A.c(1.5), wq, we).astype(A.t)
    t = A.add(y, g.k0)
    t = A.fma(g.k1, w, t)
    t = A.fma(g.k2, wn, t)
    s = A.fma(g.k4, wn, A.mul(g.k3, w))
    y = A.fma(A.sqrt(s), z1l, t)
    return y, wn


def evaluate(p, opt_type, n_steps, seed, first, n, bumps=False, dtype=np.float32, rng=None,
             fixings=None, bump_sizes=oracle.Bumps()):
    """One evaluation of the kernel's QE formulation; records [n, 14]."""
    A = _Arith(dtype, rng)
    N = n_steps
    asian, geo = opt_type in (2, 3, 4, 5), opt_type in (4, 5)
    call = opt_type in (0, 2, 4)
    fix = np.zeros(N + 1, bool)
    if fixings is None:
        fix[1:] = True
    else:
        fix[np.asarray(fixings)] = True
    n_fix = int(fix.sum()) if asian else 1
    hS, hv = bump_sizes.S0_rel * p.S0, bump_sizes.v0_rel * p.v0
    hr, hT = bump_sizes.r_abs, bump_sizes.T_abs
    dts = {"b": p.T / N, "u": (p.T + hT) / N, "d": (p.T - hT) / N}
    grids = {k: _Grid(A, p, dt) for k, dt in dts.items()}
    # scenario states: base, v0+, v0-, T+, T-
    sc = [("b", p.v0), ("b", p.v0 + hv), ("b", p.v0 - hv), ("u", p.v0), ("d", p.v0)]
    if not bumps:
        sc = sc[:1]
    ys = [np.zeros(n, dtype) for _ in sc]
    ws = [np.full(n, A.c(v0 * dts[k]), dtype) for k, v0 in sc]
    As = [np.zeros(n, dtype) for _ in sc]
    Bs, Cs, Ds = np.zeros(n, dtype), np.zeros(n, dtype), np.zeros(n, dtype)
    for j in range(N):
        q = _draws(seed, first, n, j)
        ua, ub, uv = (_uniform(q[:, k]).astype(dtype) for k in range(3))
        rad = A.sqrt(A.mul(A.c(-2.0 * LN2), A.log2(ua)))
        zs = A.mul(rad, A.cos_rev(ub))
        zv = A.mul(rad, A.sin_rev(ub))
        z1l = A.mul(zs, A.c(LOG2E))
        for i, (k, _) in enumerate(sc):
            ys[i], ws[i] = _step(A, grids[k], ys[i], ws[i], z1l, zv, uv)
        if asian and fix[j + 1]:
            for i, (k, _) in enumerate(sc):
                if geo:
                    As[i] = A.add(As[i], ys[i])
                    continue
                t = (j + 1) * dts[k]
                e = A.exp2(ys[i])
                As[i] = A.fma(A.c(math.exp(p.r * t)), e, As[i])
                if i == 0:
                    Bs = A.fma(A.c(t * math.exp(p.r * t)), e, Bs)
                    Cs = A.fma(A.c(t * t * math.exp(p.r * t)), e, Cs)
                    if dtype == np.float64:
                        Ds = A.fma(A.c(t ** 3 * math.exp(p.r * t)), e, Ds)
    return _epilogue(p, N, fix, n_fix, dts, ys, ws, As, (Bs, Cs, Ds), bumps, (hS, hv, hr, hT),
                     asian, geo, call)


def _epilogue(p, N, fix, n_fix, dts, ys, ws, As, BCD, bumps, h, asian, geo, call):
    """FP64 payoffs and estimators, as the kernel forms them from (y, w, A) and
    the weighted sums B, C, D of the base scenario (D only in FP64)."""
    Bs, Cs, Ds = BCD
    hS, hv, hr, hT = h
    n = ys[0].shape[0]
    inv_nfix = 1.0 / n_fix
    D = math.exp(-p.r * p.T)
    steps = np.nonzero(fix)[0]
    step_sum = float(steps.sum())

    def pay(Dd, X):
        inn = X - p.K if call else p.K - X
        return np.where(inn > 0.0, Dd * inn, 0.0)

    def rel_of(i, T_, dt):
        yv, av = ys[i].astype(np.float64), As[i].astype(np.float64)
        if geo:
            return np.exp((av * LN2 + p.r * dt * step_sum) * inv_nfix)
        if asian:
            return av * inv_nfix
        return np.exp(yv * LN2 + p.r * T_)

    out = np.full((n, 14), np.nan)
    x = ys[0].astype(np.float64) * LN2 + p.r * p.T
    ST = p.S0 * np.exp(x)
    rel = rel_of(0, p.T, dts["b"])
    X = p.S0 * rel
    sgn = 1.0 if call else -1.0
    itm = sgn * (X - p.K) > 0.0
    out[:, 0] = ST
    out[:, 1] = ws[0].astype(np.float64) / dts["b"]
    out[:, 2] = X
    out[:, 3] = pay(D, X)
    out[:, 4] = np.where(itm, sgn * D * rel, 0.0)
    if asian:
        dBr = rel * dts["b"] * step_sum if geo else Bs.astype(np.float64)
        out[:, 5] = np.where(itm, D * (sgn * p.S0 * dBr * inv_nfix - p.T * sgn * (X - p.K)), 0.0)
    else:
        out[:, 5] = np.where(itm, sgn * D * p.K * p.T, 0.0)
    if not bumps:
        return out
    out[:, 6] = pay(D, (p.S0 + hS) * rel)
    out[:, 7] = pay(D, (p.S0 - hS) * rel)
    out[:, 8] = pay(D, p.S0 * rel_of(1, p.T, dts["b"]))
    out[:, 9] = pay(D, p.S0 * rel_of(2, p.T, dts["b"]))
    if geo:
        tb = dts["b"] * step_sum * inv_nfix
        Xu, Xd = X * math.exp(hr * tb), X * math.exp(-hr * tb)
    elif asian:
        a, b, c, d3 = (v.astype(np.float64) for v in (As[0], Bs, Cs, Ds))
        even, odd = a + 0.5 * hr * hr * c, hr * b + hr * hr * hr / 6.0 * d3
        Xu, Xd = p.S0 * (even + odd) * inv_nfix, p.S0 * (even - odd) * inv_nfix
    else:
        Xu, Xd = ST * math.exp(hr * p.T), ST * math.exp(-hr * p.T)
    out[:, 10] = pay(math.exp(-(p.r + hr) * p.T), Xu)
    out[:, 11] = pay(math.exp(-(p.r - hr) * p.T), Xd)
    Tu, Td = p.T + hT, p.T - hT
    out[:, 12] = pay(math.exp(-p.r * Tu), p.S0 * rel_of(3, Tu, dts["u"]))
    out[:, 13] = pay(math.exp(-p.r * Td), p.S0 * rel_of(4, Td, dts["d"]))
    return out


def spread(p, opt_type, n_steps, seed, first, n, reference, bumps=False, members=8, fixings=None):
    """Per path and column, the largest |evaluation - reference| over the
    round-to-nearest evaluation and an ensemble of ``members`` Monte-Carlo-
    arithmetic binary32 evaluations (seeded, so reproducible).  ``reference``
    holds the first k record columns of the same paths (k <= 14)."""
    k = reference.shape[1]

    def dist(rng):
        v = evaluate(p, opt_type, n_steps, seed, first, n, bumps, rng=rng, fixings=fixings)
        return np.abs(v[:, :k] - reference)

    e = dist(None)
    for m in range(members):
        e = np.fmax(e, dist(np.random.default_rng(1000 + m)))
    return e
