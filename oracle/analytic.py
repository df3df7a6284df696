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
