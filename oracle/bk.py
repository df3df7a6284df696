"""Broadie-Kaya exact simulation of the Heston model -- TEST INFRASTRUCTURE (oracle).

Follows the paper's algorithm "Broadie and Kaya exact simulation algorithm"
(section "Heston Model Exact simulation") and its bottleneck sections, with the
readings where the printed formulas are garbled:

1. V_t given V_u (section "Sampling V_t from V_u"): a scaled non-central
   chi-square, V_t = c chi'^2_d(lambda) with c = sigma^2 (1 - e^{-kappa D}) / (4 kappa),
   d = 4 kappa theta / sigma^2 (the paper never defines d), and non-centrality
   lambda = V_u e^{-kappa D} / c (the printed lambda lacks its V_u factor).  For
   d > 1 the paper's decomposition chi'^2_d(lambda) = chi^2_{d-1} + (Z + sqrt(lambda))^2
   with chi^2_{d-1} = 2 Gamma((d-1)/2); for d <= 1 the Poisson mixture
   chi^2_{d + 2N}, N ~ Poisson(lambda/2).
2. The integral of V over (u, t) given V_u, V_t (section "Sampling from the
   distribution of int V"): its characteristic function Phi(a) as printed, with
   every exponent negative (e^{-kappa D} and e^{-gamma D} throughout) and the
   parentheses balanced; the modified Bessel function I_{d/2-1} of complex
   argument is kept continuous in a by counting how often the argument's phase
   winds past pi (I_nu(z e^{2 pi i m}) = e^{2 pi i m nu} I_nu(z)).  Its CDF
   F(x) = (2/pi) int_0^inf sin(ux)/u Re Phi(u) du is evaluated by the trapezoid
   rule on the grid u_j = j h, h = pi / u_eps (no aliasing for x <= u_eps), and
   inverted by bisection refined with Newton steps (the derivative of the
   trapezoid sum is its density).
3. int sqrt(V) dW2 = (V_t - V_u - kappa theta D + kappa int V) / sigma (eq. broadie_alg).
4. ln S_t = ln S_u + r D - int V / 2 + rho int sqrt(V) dW2 + sqrt(1 - rho^2) sqrt(int V) Z.

Uniforms, normals, gammas and Poisson counts come from a seeded numpy
Generator (library primitives); nothing here is shared with the GPU path.
"""
from __future__ import annotations

import math

import numpy as np
from scipy import special

from . import Params


def sample_vt(p: Params, vu: np.ndarray, dt: float, rng: np.random.Generator) -> np.ndarray:
    """V_t given V_u, a scaled non-central chi-square."""
    e = math.exp(-p.kappa * dt)
    c = p.sigma ** 2 * (1.0 - e) / (4.0 * p.kappa)
    d = 4.0 * p.kappa * p.theta / p.sigma ** 2
    lam = vu * e / c
    if d > 1.0:
        chi = 2.0 * rng.gamma((d - 1.0) / 2.0, size=vu.shape)
        z = rng.standard_normal(vu.shape)
        x = chi + (z + np.sqrt(lam)) ** 2
    else:
        n = rng.poisson(lam / 2.0)
        x = 2.0 * rng.gamma((d + 2.0 * n) / 2.0)
    return c * x


class IntegratedVariance:
    """Conditional law of int_u^t V ds given (V_u, V_t): characteristic function and CDF."""

    def __init__(self, p: Params, dt: float):
        self.p, self.dt = p, dt
        self.nu = 2.0 * p.kappa * p.theta / p.sigma ** 2 - 1.0  # d/2 - 1

    def log_phi(self, a: np.ndarray, vu: float, vt: float) -> np.ndarray:
        """log Phi(a) along an increasing grid a >= 0 (continuous branch)."""
        p, D, nu = self.p, self.dt, self.nu
        a = np.asarray(a, dtype=np.float64)
        g = np.sqrt(p.kappa ** 2 - 2.0 * p.sigma ** 2 * 1j * a)
        ek, eg = math.exp(-p.kappa * D), np.exp(-g * D)
        s2 = p.sigma ** 2
        t1 = np.log(g) - 0.5 * (g - p.kappa) * D + math.log(1.0 - ek) \
            - math.log(p.kappa) - np.log(1.0 - eg)
        t2 = (vu + vt) / s2 * (p.kappa * (1.0 + ek) / (1.0 - ek) - g * (1.0 + eg) / (1.0 - eg))
        r = math.sqrt(vu * vt)
        # ln of z(a) = 4 g e^{-g D/2} / (sigma^2 (1 - e^{-g D})) (times r), summed
        # from its factors: no underflow where e^{-g D/2} would vanish, and its
        # imaginary part is an argument of z continuous along a >= 0 (zero at
        # a = 0: arg g, -Im(g) D/2 and arg(1 - e^{-g D}) each vary
        # continuously, the last with 1 - e^{-g D} in the right half-plane)
        lz0 = np.log(4.0 * g) - 0.5 * g * D - np.log(s2 * (1.0 - eg))
        lk0 = math.log(4.0 * p.kappa) - 0.5 * p.kappa * D - math.log(s2 * (1.0 - ek))
        if r == 0.0:
            # I_nu(z) ~ (z/2)^nu / Gamma(nu+1) as z -> 0: the ratio is (z_g / z_k)^nu
            return t1 + t2 + nu * (lz0 - lk0)
        lzg, lzk = math.log(r) + lz0, math.log(r) + lk0
        zg, zk = np.exp(lzg), math.exp(lzk)

        def log_i(lz, z):
            # ln I_nu(z) on the branch of lz: the principal value of ive (scaled
            # by e^{-|Re z|}) plus nu times the turns of Im lz beyond arg z; below
            # |z| = 1e-30 the leading term of the series
            z = np.asarray(z)
            small = np.abs(z) < 1e-30
            zs = np.where(small, 1.0, z)
            turns = np.imag(lz) - np.angle(zs)
            big = np.log(special.ive(nu, zs)) + np.abs(zs.real) + 1j * nu * turns
            return np.where(small, nu * (lz - math.log(2.0)) - special.gammaln(nu + 1.0), big)

        return t1 + t2 + log_i(lzg, zg) - log_i(lzk, zk).real

    def moments(self, vu: float, vt: float):
        """Conditional mean and standard deviation from log Phi near 0:
        log Phi(a) = i mu a - s^2 a^2 / 2 + O(a^3), by Richardson on a = h, 2h."""
        guess = max(0.5 * (vu + vt) * self.dt, 1e-10)
        h = 1e-3 / guess
        lp = self.log_phi(np.array([h, 2 * h]), vu, vt)
        mu = (8.0 * lp[0].imag - lp[1].imag) / (6.0 * h)
        var = -(16.0 * lp[0].real - lp[1].real) / (6.0 * h * h)
        return mu, math.sqrt(max(var, (1e-3 * mu) ** 2))

    def cdf_grid(self, vu: float, vt: float, m_sd: float = 12.0, eps: float = 1e-10):
        """(h, u_eps, Re Phi on the grid u_j = j h, j = 1..J)."""
        mu, sd = self.moments(vu, vt)
        u_eps = mu + m_sd * sd
        h = math.pi / u_eps
        J = 64
        while True:
            a = h * np.arange(1, J + 1)
            phi = np.exp(self.log_phi(a, vu, vt))
            if abs(phi[-1]) / J < math.pi * eps / 2 or J >= 1 << 16:
                break
            J *= 2
        k = int(np.nonzero(np.abs(phi) / np.arange(1, J + 1) >= math.pi * eps / 2)[0].max()) + 1 \
            if np.any(np.abs(phi) / np.arange(1, J + 1) >= math.pi * eps / 2) else 1
        return h, u_eps, phi[:k].real

    @staticmethod
    def cdf(x, h, re_phi):
        j = np.arange(1, re_phi.size + 1)
        return h * x / math.pi + (2.0 / math.pi) * np.sum(np.sin(h * j * x) / j * re_phi)

    @staticmethod
    def pdf(x, h, re_phi):
        j = np.arange(1, re_phi.size + 1)
        return h / math.pi + (2.0 * h / math.pi) * np.sum(np.cos(h * j * x) * re_phi)

    def sample(self, vu: float, vt: float, u: float) -> float:
        """Inverse CDF at u: bisection bracket, Newton refinement."""
        h, ueps, rp = self.cdf_grid(vu, vt)
        lo, hi = 0.0, ueps
        x = min(max(self.moments(vu, vt)[0], 1e-12), ueps)
        for _ in range(200):
            f = self.cdf(x, h, rp) - u
            if abs(f) < 1e-13:
                return x
            if f > 0:
                hi = x
            else:
                lo = x
            if hi - lo < 1e-14 * max(1.0, hi):
                return x
            d = self.pdf(x, h, rp)
            xn = x - f / d if d > 0 else 0.5 * (lo + hi)
            x = xn if lo < xn < hi else 0.5 * (lo + hi)
        return x


def simulate(p: Params, times, n_paths: int, seed: int):
    """S at the given times (increasing, > 0) for n_paths exact paths: [n_paths, len(times)]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    S = np.full(n_paths, p.S0)
    V = np.full(n_paths, p.v0)
    out = np.empty((n_paths, len(times)))
    t_prev = 0.0
    for k, t in enumerate(times):
        dt = t - t_prev
        iv = IntegratedVariance(p, dt)
        vt = sample_vt(p, V, dt, rng)
        u = rng.uniform(size=n_paths)
        I = np.array([iv.sample(V[i], vt[i], u[i]) for i in range(n_paths)])
        isq = (vt - V - p.kappa * p.theta * dt + p.kappa * I) / p.sigma
        z = rng.standard_normal(n_paths)
        lnS = np.log(S) + p.r * dt - 0.5 * I + p.rho * isq \
            + math.sqrt(1.0 - p.rho ** 2) * np.sqrt(np.maximum(I, 0.0)) * z
        S = np.exp(lnS)
        V = vt
        out[:, k] = S
        t_prev = t
    return out


def price(p: Params, asian: bool, n_paths: int, seed: int, times=None, control_variate=True):
    """Discounted call price (value, std err); the Asian averages S at `times`.

    With control_variate, the payoff is regressed on its underlying X (S_T, or
    the average), whose mean is known exactly: S0 e^{rT}, or the mean of
    S0 e^{r t_i}."""
    times = tuple(times) if times is not None else (p.T,)
    S = simulate(p, times, n_paths, seed)
    X = S.mean(axis=1) if asian else S[:, -1]
    D = math.exp(-p.r * p.T)
    y = D * np.maximum(X - p.K, 0.0)
    if control_variate:
        EX = p.S0 * np.mean(np.exp(p.r * np.array(times))) if asian else p.S0 * math.exp(p.r * p.T)
        c = np.cov(y, X)
        b = c[0, 1] / c[1, 1]
        y = y - b * (X - EX)
    return float(y.mean()), float(y.std(ddof=1) / math.sqrt(n_paths))


# --------------------------------------------------------------------------
# Counter-based random inputs, for parity with the device sampler.  Block k of
# exact step j of path p is Philox4x32-10 at counter (j, lo32 p, hi32 p,
# 5 + 256 k) under key (lo32 seed, hi32 seed); a word w maps to the uniform
# ((w >> 9) + 1/2) 2^-23.  Block 0: Box-Muller of words 0, 1 gives (Zv, Zs)
# -- Zv enters the non-central chi-square, Zs the log-price -- word 2 the
# uniform of the integrated-variance inversion, word 3 the uniform of the
# Poisson count (d <= 1).  Blocks 1, 2, ...: attempt k of the gamma sampler
# (the first Box-Muller normal of words 0, 1 and the acceptance uniform of
# word 2); word 3 of block 1 is the uniform that lowers a shape below one.

BK_TAG = 5
MAX_GAMMA_ATTEMPTS = 64
MAX_POISSON_MEAN = 700.0


def _u(w) -> float:
    return ((int(w) >> 9) + 0.5) * 2.0 ** -23


def draw_block(seed: int, path: int, step: int, k: int) -> np.ndarray:
    from . import philox
    ctr = [[step, path & 0xFFFFFFFF, path >> 32, BK_TAG + (k << 8)]]
    key = [[seed & 0xFFFFFFFF, seed >> 32]]
    return philox(np.array(ctr, dtype=np.uint32), np.array(key, dtype=np.uint32))[0]


def _box_muller(w0, w1):
    r = math.sqrt(-2.0 * math.log(_u(w0)))
    a = 2.0 * math.pi * _u(w1)
    return r * math.cos(a), r * math.sin(a)


def gamma_counter(alpha: float, seed: int, path: int, step: int) -> float:
    """Gamma(alpha, 1) by Marsaglia and Tsang (ACM TOMS 26(3), 2000): with
    d = a - 1/3, c = 1/sqrt(9 d), a normal x and v = (1 + c x)^3 > 0, accept d v
    when ln U < x^2/2 + d - d v + d ln v (the full test, no squeeze).  For
    alpha < 1, a = alpha + 1 and the draw is multiplied by U^(1/alpha).
    NaN after MAX_GAMMA_ATTEMPTS rejections."""
    a = alpha + 1.0 if alpha < 1.0 else alpha
    d = a - 1.0 / 3.0
    c = 1.0 / math.sqrt(9.0 * d)
    g = math.nan
    boost = None
    for k in range(1, MAX_GAMMA_ATTEMPTS + 1):
        w = draw_block(seed, path, step, k)
        if k == 1:
            boost = _u(w[3])
        x = _box_muller(w[0], w[1])[0]
        v = 1.0 + c * x
        if v <= 0.0:
            continue
        v = v * v * v
        if math.log(_u(w[2])) < 0.5 * x * x + d - d * v + d * math.log(v):
            g = d * v
            break
    if alpha < 1.0:
        g *= boost ** (1.0 / alpha)
    return g


def poisson_inverse(mu: float, u: float) -> float:
    """Smallest k with u <= P(N <= k), N ~ Poisson(mu), by summing the
    probabilities upwards from k = 0; NaN for mu above MAX_POISSON_MEAN."""
    if mu > MAX_POISSON_MEAN:
        return math.nan
    k, pk = 0, math.exp(-mu)
    F = pk
    cap = int(mu + 40.0 * math.sqrt(mu) + 100.0)
    while u > F and k < cap:
        k += 1
        pk *= mu / k
        F += pk
    return float(k)


def sample_vt_counter(p: Params, vu: float, dt: float, seed: int, path: int, step: int):
    """V_t given V_u on the counter-based inputs; also returns (Zs, U) of block 0."""
    e = math.exp(-p.kappa * dt)
    c = p.sigma ** 2 * (1.0 - e) / (4.0 * p.kappa)
    d = 4.0 * p.kappa * p.theta / p.sigma ** 2
    lam = vu * e / c
    w = draw_block(seed, path, step, 0)
    zv, zs = _box_muller(w[0], w[1])
    if d > 1.0:
        x = 2.0 * gamma_counter(0.5 * (d - 1.0), seed, path, step) + (zv + math.sqrt(lam)) ** 2
    else:
        n = poisson_inverse(0.5 * lam, _u(w[3]))
        x = 2.0 * gamma_counter(0.5 * d + n, seed, path, step) if n == n else math.nan
    return c * x, zs, _u(w[2])


def simulate_counter(p: Params, opt_type: int, n_steps: int, seed: int, first: int = 0,
                     n_paths: int = 1, fixings=None, integral: bool = False):
    """Exact paths on the counter-based inputs: records [n_paths, 6] = (S_T, V_T,
    X, pay, pw_delta, pw_rho) as oracle.simulate, over n_steps exact steps of
    T / n_steps (the fixing dates are steps, as there).  With `integral`, also
    the integral of V over [0, T] per path."""
    from . import ASIAN_CALL, EURO_CALL, GEO_ASIAN_CALL, GEO_ASIAN_PUT
    N = n_steps
    D = p.T / N
    fix = set(range(1, N + 1)) if fixings is None else set(int(f) for f in fixings)
    asian = opt_type >= 2
    geo = opt_type in (GEO_ASIAN_CALL, GEO_ASIAN_PUT)
    call = opt_type in (EURO_CALL, ASIAN_CALL, GEO_ASIAN_CALL)
    n_fix = len(fix) if asian else 1
    iv = IntegratedVariance(p, D)
    disc = math.exp(-p.r * p.T)
    out = np.empty((n_paths, 6))
    total = np.zeros(n_paths)
    for i in range(n_paths):
        path = first + i
        x, V, A, B = 0.0, p.v0, 0.0, 0.0
        for j in range(N):
            vt, zs, uI = sample_vt_counter(p, V, D, seed, path, j)
            I = iv.sample(V, vt, uI) if vt == vt else math.nan
            total[i] += I
            isq = (vt - V - p.kappa * p.theta * D + p.kappa * I) / p.sigma
            x += p.r * D - 0.5 * I + p.rho * isq \
                + math.sqrt(1.0 - p.rho ** 2) * math.sqrt(max(I, 0.0)) * zs
            V = vt
            if asian and (j + 1) in fix:
                t = (j + 1) * D
                if geo:
                    A += math.log(p.S0) + x
                    B += t
                else:
                    S = p.S0 * math.exp(x)
                    A += S
                    B += t * S
        S = p.S0 * math.exp(x)
        X = math.exp(A / n_fix) if geo else A / n_fix if asian else S
        if geo:
            B = X * B
        sgn = 1.0 if call else -1.0
        itm = sgn * (X - p.K) > 0.0
        pay = disc * sgn * (X - p.K) if itm else 0.0
        dpw = sgn * disc * X / p.S0 if itm else 0.0
        if asian:
            rpw = disc * (sgn * B / n_fix - p.T * sgn * (X - p.K)) if itm else 0.0
        else:
            rpw = sgn * disc * p.K * p.T if itm else 0.0
        out[i] = (S, V, X, pay, dpw, rpw)
    return (out, total) if integral else out
