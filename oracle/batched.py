"""Per-block tolerance-driven compression for the batched workload.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Each block K (m_b x n_b) is compressed to a relative spectral tolerance eps
by the given-tolerance scheme of Sections 12-14, in this order:

1. Draw l0 Gaussian columns (block's own stream) and r probe vectors
   (Section 14; r = 10, alpha = 1/10).
2. Q = orth(K Omega) (Figure 1 / Figure 13 with l0 vectors), B = Q^T K.
3. Certificate of the pair (Q, B): bound = 10 sqrt(2/pi) max_i ||(K - Q B) g_i||.
   sigma_hat_1 = largest singular value of B.
4. While bound > eps sigma_hat_1 / 2 and the rank can grow by b: draw the next b
   Gaussian columns (continuing Omega), Y = (I - QQ^T)^2 K G, Q_new = orth(Y),
   B_new = Q_new^T K, append (Figure 12 with the residual applied implicitly).
5. SVD of B; keep the singular values above eps sigma_hat_1 / 2.  Then
   ||K - U S V^T|| <= bound + sigma_{kept+1}(B) <= eps sigma_hat_1 with the
   certificate's probability.

Per-block streams of the counter-based generator: 16*blk + 4 for Omega and
its continuation, 16*blk + 6 for the probes.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

from . import philox
from .rsvd import orth, svd_small


@dataclass
class BlockResult:
    U: np.ndarray
    S: np.ndarray
    V: np.ndarray
    rank: int          # columns kept after truncation
    basis: int         # width of the certified basis
    bound: float
    sigma1: float
    certified: bool


def compress_block(K: np.ndarray, eps: float, seed: int, blk: int, l0: int = 16, b: int = 8, r: int = 10,
                   rank_cap: int = 64) -> BlockResult:
    K = np.asarray(K, dtype=np.float64)
    m, n = K.shape
    s_omega, s_probe = 16 * blk + 4, 16 * blk + 6
    G0 = philox.gaussian(n, l0, seed, s_omega)
    Gc = philox.gaussian(n, r, seed, s_probe)
    Q = orth(K @ G0)
    B = Q.T @ K
    c_alpha = 10.0 * math.sqrt(2.0 / math.pi)

    def bound_of(Q_, B_):
        E = K @ Gc - Q_ @ (B_ @ Gc)
        return c_alpha * float(np.max(np.linalg.norm(E, axis=0)))

    bound = bound_of(Q, B)
    sigma1 = float(np.linalg.svd(B, compute_uv=False)[0])
    steps = 0
    cap = min(rank_cap, m, n)
    while bound > 0.5 * eps * sigma1 and Q.shape[1] + b <= cap:
        Gb = philox.gaussian(n, b, seed, s_omega, col0=l0 + steps * b)
        Y = K @ Gb
        Y = Y - Q @ (Q.T @ Y)
        Y = Y - Q @ (Q.T @ Y)
        Qn = orth(Y)
        Q = np.column_stack([Q, Qn])
        B = np.vstack([B, Qn.T @ K])
        bound = bound_of(Q, B)
        steps += 1
    uh, d, v = svd_small(B)
    keep = int(np.sum(d > 0.5 * eps * sigma1))
    keep = max(keep, 1)
    return BlockResult((Q @ uh)[:, :keep], d[:keep], v[:, :keep], keep, Q.shape[1], bound, sigma1,
                       bound <= 0.5 * eps * sigma1)
