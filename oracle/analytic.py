"""Closed-form and semi-analytic references -- TEST INFRASTRUCTURE (oracle).

- Heston European prices from the characteristic function of ln S_T, written
  in the "little trap" form of Albrecher, Mayer, Schoutens and Tistaert (2007)
  so that the complex logarithm stays on its principal branch; prices by the
  Gil-Pelaez inversion (probabilities P1, P2) and, independently, by Lewis'
  single-integral formula.  The model is the paper's Heston SDE pair (Heston
  Model for option pricing, eq. heston_eq) under the risk-neutral measure
  (Background, risk-neutral pricing).
- Greeks: Delta = P1 and Rho = K T exp(-rT) P2 in closed form; Gamma,
  sensitivities to v0, T, kappa, theta, sigma, rho by Richardson-extrapolated
  central differences of the Gil-Pelaez price.
- Black-Scholes call and put prices and Greeks.
"""
from __future__ import annotations

import math
import warnings

import numpy as np
from scipy import integrate
from scipy.special import ndtr

from . import Params


def heston_cf(u, p: Params, T: float | None = None):
    """E[exp(i u ln S_T)] under Heston (little-trap form); u may be complex."""
    T = p.T if T is None else T
    u = np.asarray(u, dtype=np.complex128)
    iu = 1j * u
    k, th, s, rho = p.kappa, p.theta, p.sigma, p.rho
    b = k - rho * s * iu
    d = np.sqrt(b * b + s * s * (iu + u * u))
    g = (b - d) / (b + d)
    e = np.exp(-d * T)
    C = (k * th / (s * s)) * ((b - d) * T - 2.0 * np.log((1.0 - g * e) / (1.0 - g)))
    D = ((b - d) / (s * s)) * (1.0 - e) / (1.0 - g * e)
    return np.exp(iu * (math.log(p.S0) + p.r * T) + C + D * p.v0)


def _quad(f):
    with warnings.catch_warnings():
        # quad reports round-off once the integrand is resolved to ~1e-13
        warnings.simplefilter("ignore", integrate.IntegrationWarning)
        val, _ = integrate.quad(f, 0.0, np.inf, epsabs=1e-12, epsrel=1e-12, limit=2000)
    return val


def probabilities(p: Params):
    """Gil-Pelaez P1 (share measure) and P2 (risk-neutral) of S_T > K."""
    lnK = math.log(p.K)
    phi_mi = heston_cf(-1j, p)  # = S0 exp(rT)

    def f1(u):
        return (np.exp(-1j * u * lnK) * heston_cf(u - 1j, p) / (1j * u * phi_mi)).real

    def f2(u):
        return (np.exp(-1j * u * lnK) * heston_cf(u, p) / (1j * u)).real

    P1 = 0.5 + _quad(f1) / math.pi
    P2 = 0.5 + _quad(f2) / math.pi
    return P1, P2


def heston_call(p: Params) -> float:
    P1, P2 = probabilities(p)
    return p.S0 * P1 - p.K * math.exp(-p.r * p.T) * P2


def heston_put(p: Params) -> float:
    """By put-call parity of the exact model: P = C - S0 + K exp(-rT)."""
    return heston_call(p) - p.S0 + p.K * math.exp(-p.r * p.T)


def heston_call_lewis(p: Params) -> float:
    """Lewis (2001): C = S0 - sqrt(S0 K) e^{-rT/2}/pi int Re[e^{iuk} psi(u - i/2)]/(u^2+1/4) du,
    with k = ln(S0/K) + rT and psi the characteristic function of ln(S_T/S0) - rT."""
    k = math.log(p.S0 / p.K) + p.r * p.T
    shift = math.log(p.S0) + p.r * p.T

    def f(u):
        z = u - 0.5j
        psi = heston_cf(z, p) * np.exp(-1j * z * shift)
        return (np.exp(1j * u * k) * psi).real / (u * u + 0.25)

    return p.S0 - math.sqrt(p.S0 * p.K) * math.exp(-0.5 * p.r * p.T) / math.pi * _quad(f)


def _richardson(f, x, h):
    d1 = (f(x + h) - f(x - h)) / (2 * h)
    d2 = (f(x + h / 2) - f(x - h / 2)) / h
    return (4 * d2 - d1) / 3


def heston_call_greeks(p: Params) -> dict:
    """Price and sensitivities of the European call.

    delta = P1, rho = K T e^{-rT} P2 (closed form); the rest by Richardson
    central differences of the Gil-Pelaez price.  'theta' is -dC/dT."""
    P1, P2 = probabilities(p)
    price = p.S0 * P1 - p.K * math.exp(-p.r * p.T) * P2
    out = {"price": price, "delta": P1, "rho": p.K * p.T * math.exp(-p.r * p.T) * P2}

    def d(name, h):
        return _richardson(lambda x: heston_call(p.replace(**{name: x})), getattr(p, name), h)

    out["gamma"] = _richardson(lambda s: probabilities(p.replace(S0=s))[0], p.S0, 0.01 * p.S0)
    out["vega"] = d("v0", 1e-3 * p.v0)
    out["theta"] = -d("T", 1e-3 * p.T)
    out["d_kappa"] = d("kappa", 1e-3 * p.kappa)
    out["d_theta"] = d("theta", 1e-3 * p.theta)
    out["d_sigma"] = d("sigma", 1e-3 * p.sigma)
    out["d_rho"] = d("rho", 1e-3)
    return out


# --------------------------------------------------------------------------
def bs_call(S0, K, r, T, vol):
    sd = vol * math.sqrt(T)
    d1 = (math.log(S0 / K) + (r + 0.5 * vol * vol) * T) / sd
    d2 = d1 - sd
    return S0 * ndtr(d1) - K * math.exp(-r * T) * ndtr(d2)


def bs_put(S0, K, r, T, vol):
    return bs_call(S0, K, r, T, vol) - S0 + K * math.exp(-r * T)


def bs_call_greeks(S0, K, r, T, vol):
    sd = vol * math.sqrt(T)
    d1 = (math.log(S0 / K) + (r + 0.5 * vol * vol) * T) / sd
    d2 = d1 - sd
    pdf = math.exp(-0.5 * d1 * d1) / math.sqrt(2 * math.pi)
    return {
        "price": bs_call(S0, K, r, T, vol),
        "delta": float(ndtr(d1)),
        "gamma": pdf / (S0 * sd),
        "rho": K * T * math.exp(-r * T) * float(ndtr(d2)),
    }


# --------------------------------------------------------------------------
# Discretely monitored geometric-average Asian options under Heston.
#
# ln G = (1/n) sum_i ln S_{t_i}.  Its transform E[exp(u ln G)] follows from the
# affine structure of (ln S, V): between consecutive fixing dates the
# conditional transform of the dates still to come is exp(a ln S_t + B V_t + A)
# with a constant (u times the weights of those dates) and (A, B) solving, in
# the time to the next date tau,
#     B' = sigma^2 B^2 / 2 + (rho sigma a - kappa) B + (a^2 - a) / 2,
#     A' = kappa theta B + r a,
# whose solution from B(0) = B0 is closed-form; at a fixing date a grows by
# u / n while A and B carry over.  The recursion runs backward from the last
# date to time 0.

def _riccati_step(a, B0, A0, tau, p: Params):
    """(A, B) after time tau from (A0, B0), for the coefficient a of ln S."""
    c2 = 0.5 * p.sigma * p.sigma
    c1 = p.rho * p.sigma * a - p.kappa
    c0 = 0.5 * (a * a - a)
    d = np.sqrt(c1 * c1 - 4.0 * c2 * c0)
    d = np.where(d.real < 0, -d, d)
    r2 = (-c1 - d) / (2.0 * c2)  # attracting root
    r1 = (-c1 + d) / (2.0 * c2)
    Cp = (B0 - r2) / (B0 - r1)
    e = np.exp(-d * tau)
    B = (r2 - r1 * Cp * e) / (1.0 - Cp * e)
    intB = r2 * tau - np.log((1.0 - Cp * e) / (1.0 - Cp)) / c2
    A = A0 + p.r * a * tau + p.kappa * p.theta * intB
    return A, B


def geometric_transform(u, p: Params, times):
    """E[exp(u ln G)] for complex u (array), G the geometric average of S over
    the fixing times (increasing, in (0, T])."""
    u = np.asarray(u, dtype=np.complex128)
    t = np.asarray(times, dtype=np.float64)
    n = t.size
    w = u / n
    a = w.copy()
    A = np.zeros_like(u)
    B = np.zeros_like(u)
    for k in range(n - 1, -1, -1):
        t_prev = t[k - 1] if k > 0 else 0.0
        A, B = _riccati_step(a, B, A, t[k] - t_prev, p)
        if k > 0:
            a = a + w
    return np.exp(a * math.log(p.S0) + B * p.v0 + A)


def geometric_asian_call(p: Params, times) -> float:
    """e^{-rT} E[(G - K)^+] by Gil-Pelaez inversion of the transform of ln G."""
    lnK = math.log(p.K)
    EG = geometric_transform(np.array([1.0]), p, times)[0].real

    def cf(v):
        return geometric_transform(1j * np.atleast_1d(v), p, times)

    def f1(v):
        return (np.exp(-1j * v * lnK) * geometric_transform(1j * v + 1.0, p, times)
                / (1j * v * EG)).real[0]

    def f2(v):
        return (np.exp(-1j * v * lnK) * cf(v) / (1j * v)).real[0]

    P1 = 0.5 + _quad(lambda v: f1(np.atleast_1d(v))) / math.pi
    P2 = 0.5 + _quad(f2) / math.pi
    return math.exp(-p.r * p.T) * (EG * P1 - p.K * P2)


def geometric_asian_put(p: Params, times) -> float:
    """By parity: P = C - e^{-rT} (E[G] - K)."""
    EG = geometric_transform(np.array([1.0]), p, times)[0].real
    return geometric_asian_call(p, times) - math.exp(-p.r * p.T) * (EG - p.K)


def geometric_asian_call_deterministic_variance(p: Params, times) -> float:
    """sigma = 0: the variance is deterministic, V_t = theta + (v0 - theta) e^{-kappa t},
    so ln G is normal with mean ln S0 + mean_i (r t_i - I(t_i)/2) and variance
    mean_{i,j} I(min(t_i, t_j)), I(t) = int_0^t V; Black-Scholes form."""
    t = np.asarray(times, dtype=np.float64)

    def I(x):
        return p.theta * x + (p.v0 - p.theta) * (1.0 - np.exp(-p.kappa * x)) / p.kappa

    mu = math.log(p.S0) + float(np.mean(p.r * t - 0.5 * I(t)))
    var = float(np.mean(I(np.minimum.outer(t, t))))
    sd = math.sqrt(var)
    d1 = (mu - math.log(p.K) + var) / sd
    d2 = d1 - sd
    return math.exp(-p.r * p.T) * (math.exp(mu + 0.5 * var) * ndtr(d1) - p.K * ndtr(d2))
