"""Rounding sensitivity of the oracle's pathwise derivatives -- test infrastructure.

The oracle's forward-mode derivatives of a Milstein path (``oracle.tangent``)
multiply by d sqrt(V+ dt)/dV+ = sqrt(dt/V+)/2 at every step; where the
variance comes close to zero that factor is large, and so is the relative
error of V+ itself (V is a sum of terms of size theta dt or larger, so its
absolute rounding error is a few roundings of that size, not of V).  A
derivative is then as sensitive to rounding as the path's largest such
factor a_p (reported by the oracle) makes it, and more: the quantities it
multiplies are themselves uncertain in proportion.

``spread`` measures that sensitivity directly: it evaluates the oracle's
derivatives again with every normal input multiplied by (1 + xi u ulps),
xi uniform in [-1, 1] (a perturbation of each step of the size of a few
roundings in the working precision: u = 2^-53 for binary64, 2^-24 for
binary32), and returns per path and column the largest change over the
ensemble.  The parity tests of the adjoint kernels use it as the rounding
allowance of each path: where the path is well conditioned it is far below
the 1e-12 / 1e-5 bars, and where the variance touches zero it says how far
any evaluation in that precision can land.
"""
from __future__ import annotations

import numpy as np

import oracle

U = {0: 2.0 ** -53, 1: 2.0 ** -24}


def spread(p, opt_type, n_steps, seed, first, n, prec, mode=oracle.FULL_TRUNC, fixings=None,
           ulps=4.0, members=8, threads=8):
    """(tangent [n, 9] of the unperturbed normals, largest change [n, 8] of
    columns 0..7 over ``members`` perturbed evaluations)."""
    za, zb = oracle.normals(seed, first, n, n_steps)
    base = oracle.tangent(p, opt_type, n_steps, seed, first, n, mode, fixings, za=za, zb=zb,
                          threads=threads)
    s = np.zeros((n, 8))
    eps = U[prec] * ulps
    for m in range(members):
        g = np.random.default_rng(2000 + m)
        t = oracle.tangent(p, opt_type, n_steps, seed, first, n, mode, fixings,
                           za=za * (1.0 + eps * g.uniform(-1.0, 1.0, za.shape)),
                           zb=zb * (1.0 + eps * g.uniform(-1.0, 1.0, zb.shape)), threads=threads)
        s = np.fmax(s, np.abs(t[:, :8] - base[:, :8]))
    return base, s
