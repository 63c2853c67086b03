"""Inputs, labels and decision rule of the learned (p, q) selector.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The selector replaces the hand rules for the oversampling p (Section 4: p = 10
is usually enough) and the number of power steps q (Section 8: q = 1 or 2 is
typical) when a tolerance eps has to be met.

* Probe: Y16 = A G16 with a 16-column Gaussian G16 (probe stream of the
  counter-based generator); its singular values sigma_1..sigma_16 describe the
  leading part of the spectrum of A at the cost of one thin pass.
* Features (16): log10(max(sigma_{i+1} / sigma_1, 1e-12)) / 6 for
  i = 1..15, and log10(k) / 3 for the target rank k of the item.
* Grid: p in P_GRID, q in Q_GRID; output o = 8 * (index of q) + (index of p).
* Label of a grid point: 1 when the plain method (Figure 5, no growth) with
  that (p, q) returns a rank-(k+p) factorisation whose Section 14 certificate
  (10 probes, alpha = 1/10, s = 0) is <= eps * sigma_1.
* Decision: among the grid points whose predicted probability P is >= tau,
  the one of least expected time cost * (2 - P) (a miss costs about as much
  again through the fallback); if there is none, the most probable one.

Parity status: the feature map, the decision rule and the prefix labels are
pinned (scale invariance, rank revelation, brute force over the grid, the
prefix property of the re-orthonormalised power scheme); the trained
network's decisions themselves are parity unpinned (only their gain is
measured).
"""
from __future__ import annotations

import math

import numpy as np

from . import philox
from .rsvd import certificate_qb, orth

P_GRID = (0, 5, 10, 20, 40, 80, 160, 320)
Q_GRID = (0, 1, 2, 3, 4)
N_GRID = len(P_GRID) * len(Q_GRID)


def probe_sigma(A: np.ndarray, seed: int) -> np.ndarray:
    """Singular values of A G16 (descending), G16 from the probe stream."""
    A = np.asarray(A, np.float64)
    G = philox.gaussian(A.shape[1], 16, seed, philox.STREAM_PROBE)
    return np.linalg.svd(A @ G, compute_uv=False)


def features(sig16: np.ndarray, k: int) -> np.ndarray:
    s = np.asarray(sig16, np.float64)
    x = np.empty(16)
    ratio = s[1:16] / s[0] if s[0] > 0 else np.zeros(15)
    x[:15] = np.log10(np.maximum(ratio, 1e-12)) / 6.0
    x[15] = math.log10(k) / 3.0
    return x


def cost_ms(m: int, n: int, k: int, p: int, q: int) -> float:
    """Modelled time (ms) of the plain method at (p, q) on one MI355X: a
    fixed part, 2q+2 passes over A at an effective 48 TFLOP/s, 2q+1
    CholeskyQR passes and the Stage B Jacobi, fitted to measured timings."""
    l = min(k + p, m, n)
    return (0.081 + (2 * q + 2) * 2.0 * m * n * l * 20.9e-12 + (2 * q + 1) * 0.104 * max(l / 128.0, 1.0) ** 1.5
            + 1.08 * (l / 95.0) ** 1.5)


def grid_points(m: int, n: int, k: int):
    """(o, p, q) for the grid points whose l = k + p fits min(m, n) and 1024."""
    out = []
    for qi, q in enumerate(Q_GRID):
        for pi, p in enumerate(P_GRID):
            if k + p <= min(m, n, 1024):
                out.append((qi * len(P_GRID) + pi, p, q))
    return out


def choose(prob: np.ndarray, m: int, n: int, k: int, tau: float):
    """Least expected time cost * (2 - P) over the grid points with P >= tau;
    the most probable point if there is none."""
    pts = grid_points(m, n, k)
    ok = [(cost_ms(m, n, k, p, q) * (2.0 - prob[o]), o, p, q) for o, p, q in pts if prob[o] >= tau]
    if ok:
        e, o, p, q = min(ok)
        return p, q
    o, p, q = max(pts, key=lambda t: (prob[t[0]], -t[0]))
    return p, q


def plain_certificates(A: np.ndarray, k: int, q: int, seed: int, ps, n_probe: int = 10):
    """Certificate bound of the rank-(k+p) result of the plain method for each
    p in ps: a separate run of Figure 5 with the first k+p columns of the
    test matrix (same seed, same probes), by definition."""
    A = np.asarray(A, np.float64)
    n = A.shape[1]
    Gc = philox.gaussian(n, n_probe, seed, philox.STREAM_CERT)
    out = []
    for p in ps:
        l = k + p
        G = philox.gaussian(n, l, seed, philox.STREAM_OMEGA)
        Q = orth(A @ G)
        for _ in range(q):
            W = orth(A.T @ Q)
            Q = orth(A @ W)
        B = Q.T @ A
        out.append(certificate_qb(A, Q, B, Gc))
    return out
