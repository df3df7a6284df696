"""The Milstein or QE path and its forward-mode derivatives evaluated in
binary32 on the CPU -- test infrastructure.

The single-precision adjoint kernels carry a path's state (log-price,
variance, running average) and, in the reverse sweep, its adjoints in
binary32.  Where the variance comes close to zero the scheme's variance map
has a large derivative (d sqrt(V+ dt)/dV+ = sqrt(dt/V+)/2, times sigma Z2),
so a relative rounding error made at one step comes back multiplied at every
later step, and the derivatives of the payoff, which are themselves formed
from those factors, are more sensitive still.  How far any binary32
evaluation lands from the exact (FP64) result on such a path is a property of
the path, not of one evaluation order.

This module measures it.  It evaluates the same quantities as the oracle's
forward-mode derivative routine (the discounted payoff and its derivatives
with respect to S0, v0, r, kappa, theta, sigma, rho; the paper's pathwise
method extended to the model parameters) in C (``tangent_mca.c``, built with
gcc, no fast-math), in a chosen working type, and optionally with Monte Carlo
arithmetic (Parker, 1997, "Monte Carlo
Arithmetic: exploiting randomness in floating-point arithmetic"): every
operation's exact result is multiplied by (1 + xi u), xi uniform in [-1, 1],
u = 2^-24 (binary32) or 2^-53, before it is rounded to the working type.  The
normals, which a binary32 kernel computes with binary32 transcendentals, get
a relative perturbation of two roundings plus the absolute error of the
hardware sine and cosine times the Box-Muller radius.

``spread`` returns, per path and column, the largest distance from the
oracle over the round-to-nearest evaluation and an ensemble of such
evaluations.  It is neither the oracle (whose arithmetic it does not share:
it only reads the oracle's normals, the random inputs both sides consume) nor
the GPU path.  With binary64 and no perturbation it reproduces the oracle's
derivatives to 1e-13 on well-conditioned paths (a CPU test checks this),
which pins its formulas.

Under Andersen's QE scheme the same holds where the quadratic branch's
b + Zv nearly cancels (V' = a (b + Zv)^2 then carries the relative error of
Zv divided by |b + Zv|) and where a step sits close to the branch switch
psi = 3/2 or to the point mass of the exponential branch; there the inputs are
(Zs, Zv, Uv), the oracle's QE draws, and the branch decisions are taken on the
evaluation's own rounded values.

Columns: 0 payoff, 1..7 d/d(S0, v0, r, kappa, theta, sigma, rho), 8 the
Milstein path's largest d sqrt(V+ dt)/dV+ (as the oracle reports it); 0 for QE.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

import oracle

# Ensemble size and the multiple of its spread that forms the parity bar: a
# CPU test shows that 4 x the spread of 16 members covers 16 further members
# on every path of a Feller-violating case.
MEMBERS = 16
FACTOR = 4.0


_SRC = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tangent_mca.c")
_LIB = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libtangent_mca.so")
_lib = None


class _CParams(ctypes.Structure):
    _fields_ = [(k, ctypes.c_double) for k in
                ("S0", "K", "r", "T", "v0", "kappa", "theta", "sigma", "rho")]


def build(force: bool = False) -> str:
    """Compile libtangent_mca.so with gcc (plain -O2, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-Wall", "-Wextra",
                               "-o", tmp, _SRC, "-lm", "-lpthread"])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB)
        P = ctypes.POINTER
        L.tm_evaluate.argtypes = [P(_CParams), ctypes.c_int, ctypes.c_uint32, P(ctypes.c_uint8),
                                  ctypes.c_int, P(ctypes.c_double), P(ctypes.c_double),
                                  P(ctypes.c_double), ctypes.c_uint64, ctypes.c_int,
                                  ctypes.c_uint64, ctypes.c_int, P(ctypes.c_double)]
        L.tm_evaluate.restype = ctypes.c_int
        _lib = L
    return _lib


def inputs(p, opt_type, n_steps, seed, first, n, mode=oracle.FULL_TRUNC):
    """The random inputs both sides consume: (Za, Zb) for Milstein, (Zs, Zv, Uv) for QE."""
    if mode == oracle.QE:
        return oracle.qe_draws_block(seed, first, n, n_steps)
    return oracle.normals(seed, first, n, n_steps)


def evaluate(p, opt_type, n_steps, seed, first, n, mode=oracle.FULL_TRUNC, fixings=None,
             dtype=np.float32, mca_seed=0, normals=None, threads=8):
    """One evaluation in ``dtype`` (round to nearest for ``mca_seed`` 0, else
    Monte Carlo arithmetic from that seed); [n, 9] in the oracle's tangent
    layout (column 8: the Milstein path's largest sqrt(dt / V+) / 2; 0 for QE)."""
    if mode not in (oracle.FULL_TRUNC, oracle.ABSORB, oracle.QE):
        raise ValueError("the derivative path follows the Milstein or QE scheme")
    if opt_type not in (0, 1, 2, 3):
        raise ValueError("European and arithmetic-average Asian payoffs only")
    z = normals if normals is not None else inputs(p, opt_type, n_steps, seed, first, n, mode)
    z = [np.ascontiguousarray(a, np.float64) for a in z]
    assert all(a.shape == (n, n_steps) for a in z) and len(z) == (3 if mode == oracle.QE else 2)
    fix = np.zeros(n_steps + 1, np.uint8)
    if fixings is None:
        fix[1:] = 1
    else:
        fix[np.asarray(fixings)] = 1
    out = np.empty((n, 9))
    P = ctypes.POINTER
    dp = P(ctypes.c_double)
    cp = _CParams(p.S0, p.K, p.r, p.T, p.v0, p.kappa, p.theta, p.sigma, p.rho)
    scheme = {oracle.FULL_TRUNC: 0, oracle.ABSORB: 1, oracle.QE: 2}[mode]
    rc = lib().tm_evaluate(ctypes.byref(cp), opt_type, n_steps,
                           fix.ctypes.data_as(P(ctypes.c_uint8)), scheme,
                           z[0].ctypes.data_as(dp), z[1].ctypes.data_as(dp),
                           z[2].ctypes.data_as(dp) if len(z) == 3 else None, n,
                           int(dtype == np.float32), mca_seed, threads, out.ctypes.data_as(dp))
    if rc != 0:
        raise ValueError("tm_evaluate: invalid argument")
    return out


def spread(p, opt_type, n_steps, seed, first, n, reference, mode=oracle.FULL_TRUNC,
           fixings=None, dtype=np.float32, members=MEMBERS, threads=8):
    """Per path and column 0..7, the largest |evaluation - reference| over the
    round-to-nearest evaluation in ``dtype`` and ``members`` Monte-Carlo-
    arithmetic evaluations (seeds 1..members, so reproducible).
    ``reference``: the oracle's [n, >=8] derivatives of the same paths."""
    z = inputs(p, opt_type, n_steps, seed, first, n, mode)
    ref = reference[:, :8]
    e = np.zeros_like(ref)
    for m in range(members + 1):
        v = evaluate(p, opt_type, n_steps, seed, first, n, mode, fixings, dtype, m, z, threads)
        e = np.fmax(e, np.abs(v[:, :8] - ref))
    return e


def floors(p):
    """Per-column floors of the relative parity bar: S0 for the payoff and for
    d/dv0, d/dsigma, d/drho; 1 for d/dS0; K T for d/dr; S0 T for d/dkappa and
    d/dtheta."""
    return np.array([p.S0, 1.0, p.S0, p.K * p.T, p.S0 * p.T, p.S0 * p.T, p.S0, p.S0])


TOL = {np.float64: 1e-12, np.float32: 1e-5}


def bars(p, opt_type, n_steps, seed, first, n, reference, mode=oracle.FULL_TRUNC, fixings=None,
         dtype=np.float32, members=MEMBERS, threads=8):
    """Per-path parity bars [n, 8]: max(tol max(|o|, floor), FACTOR x
    ``spread``), tol 1e-12 (binary64) or 1e-5 (binary32)."""
    s = spread(p, opt_type, n_steps, seed, first, n, reference, mode, fixings, dtype, members,
               threads)
    plain = TOL[dtype] * np.maximum(np.abs(reference[:, :8]), floors(p))
    return np.maximum(plain, FACTOR * s)
