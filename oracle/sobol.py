"""Quasi-random normals for the oracle: Sobol points and a Brownian bridge.

TEST INFRASTRUCTURE (oracle).  The paper introduces Sobol low-discrepancy
sequences (section "Pseudo random number generation", Sobol sequences and
properties A/A') but never says how points are mapped to the time steps of a
path; the readings used here:

- points: the unscrambled Sobol sequence of dimension 2N in Gray-code order,
  30-bit, exactly as scipy.stats.qmc.Sobol(2N, scramble=False) draws it;
- replicates: R independent digital shifts; replicate r XORs coordinate d with
  the top 30 bits of word 0 of Philox4x32-10(counter=(d, r, 0, 1), key=seed);
  path index p = r*M + i uses point i of replicate r (M = points per replicate);
- uniforms: u = ((x XOR s) + 1/2) 2^-30, never 0 or 1; normals z = Phi^{-1}(u);
- Brownian bridge on the unit grid 0..N (one unit of variance per step):
  B_N = sqrt(N) z_0, then intervals (l, r) are taken first-in first-out
  starting from (0, N); when r - l >= 2 the midpoint m = floor((l+r)/2) gets
  B_m = ((r-m) B_l + (m-l) B_r)/(r-l) + sqrt((m-l)(r-m)/(r-l)) z_k with
  k counting nodes in that order, and (l, m), (m, r) are queued;
- node k takes coordinates 2k (the price motion Wa) and 2k+1 (Wb);
- step j's normals are Za_j = Ba_{j+1} - Ba_j and likewise Zb_j.
"""
from __future__ import annotations

import math
import warnings
from collections import deque

import numpy as np
from scipy.special import ndtri
from scipy.stats import qmc

from . import philox


def points(dim: int, first: int, n: int) -> np.ndarray:
    """Integer Sobol points (30-bit) i = first .. first+n-1, shape [n, dim]."""
    eng = qmc.Sobol(dim, scramble=False, bits=30)
    if first:
        eng.fast_forward(first)
    with warnings.catch_warnings():
        # scipy warns when n is not a power of two; slices of the sequence are intended here
        warnings.simplefilter("ignore", UserWarning)
        x = eng.random(n)
    return np.rint(x * 2.0**30).astype(np.uint64)


def shifts(dim: int, replicates: int, seed: int) -> np.ndarray:
    """Digital shifts [replicates, dim] (30-bit)."""
    d = np.arange(dim, dtype=np.uint32)
    out = np.empty((replicates, dim), dtype=np.uint64)
    key = np.array([[seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF]], dtype=np.uint32)
    for r in range(replicates):
        ctr = np.stack([d, np.full_like(d, r), np.zeros_like(d), np.ones_like(d)], axis=1)
        w = philox(ctr, np.repeat(key, dim, axis=0))
        out[r] = (w[:, 0] >> 2).astype(np.uint64)
    return out


def bridge_plan(n_steps: int):
    """Bridge nodes in construction order: list of (m, l, r); the first is (N, 0, None)."""
    plan = [(n_steps, 0, None)]
    q = deque([(0, n_steps)])
    while q:
        l, r = q.popleft()
        if r - l >= 2:
            m = (l + r) // 2
            plan.append((m, l, r))
            q.append((l, m))
            q.append((m, r))
    return plan


def bridge(z: np.ndarray) -> np.ndarray:
    """Unit-grid Brownian bridge: z [n, N] standard normals in node order ->
    increments [n, N] (standard normals in time order)."""
    n, N = z.shape
    B = np.zeros((n, N + 1))
    for k, (m, l, r) in enumerate(bridge_plan(N)):
        if r is None:
            B[:, m] = math.sqrt(N) * z[:, k]
        else:
            B[:, m] = ((r - m) * B[:, l] + (m - l) * B[:, r]) / (r - l) \
                + math.sqrt((m - l) * (r - m) / (r - l)) * z[:, k]
    return np.diff(B, axis=1)


def uniforms(n_steps: int, first_path: int, n_paths: int, replicates: int,
             points_per_replicate: int, seed: int) -> np.ndarray:
    """Shifted uniforms [n_paths, 2N] for paths first_path .. (coordinate order)."""
    dim = 2 * n_steps
    sh = shifts(dim, replicates, seed)
    out = np.empty((n_paths, dim))
    p = first_path
    row = 0
    while row < n_paths:
        r, i = divmod(p, points_per_replicate)
        take = min(n_paths - row, points_per_replicate - i)
        x = points(dim, i, take) ^ sh[r][None, :]
        out[row:row + take] = (x.astype(np.float64) + 0.5) * 2.0**-30
        row += take
        p += take
    return out


def normals(n_steps: int, first_path: int, n_paths: int, replicates: int,
            points_per_replicate: int, seed: int):
    """Quasi-random (Za, Zb), each [n_paths, N], through the Brownian bridge."""
    u = uniforms(n_steps, first_path, n_paths, replicates, points_per_replicate, seed)
    z = ndtri(u)
    za = bridge(z[:, 0::2])
    zb = bridge(z[:, 1::2])
    return za, zb
