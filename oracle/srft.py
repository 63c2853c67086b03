"""Structured random sketch of Section 6: Omega = D F S.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Section 6 replaces the Gaussian test matrix of Figure 1 by a product of a
random diagonal D, a fast unitary transform F and a column subsampling S,
so that Y = A Omega costs O(m n log l) instead of O(m n l); Section 14,
item (1), pairs it with the Gaussian-probe certificate.  The paper states
the transform as the complex DFT and allows other fast transforms.  The
reading here, in real arithmetic (the library handles real matrices only):

  N      = 2^ceil(log2 n)  (rows of A's row space padded with zeros to N)
  D      = diag(d_0 .. d_{N-1}), d_i = +1 or -1 (the real unit circle)
  F      = H_N / sqrt(N), H_N the Sylvester-Hadamard matrix,
           H_N(i, k) = (-1)^popcount(i & k)  (orthogonal after scaling)
  S      = columns s_0 .. s_{l-1} of the N x N identity, distinct, drawn
           without replacement
  Omega  = the first n rows of D F S  (n x l)

Random numbers come from the counter-based generator of ``oracle.philox``
(key = seed), stream ``STREAM_SRHT``:
  signs:  word w = i mod 4 of Philox(counter = (i div 4, 0, STREAM_SRHT, 0));
          d_i = -1 if its lowest bit is 1, else +1
  subset: the first l steps of a Fisher-Yates shuffle of 0 .. N-1: with
          perm = identity, for j = 0 .. l-1,
            u_j = word (j mod 4) of Philox(counter = (j div 4, 1, STREAM_SRHT, 0))
            r   = j + floor(u_j (N - j) / 2^32)
            swap perm[j], perm[r]
          s_j = perm[j]
"""
from __future__ import annotations

import math

import numpy as np

from . import philox
from .rsvd import orth, stage_b

STREAM_SRHT = 10


def padded_size(n: int) -> int:
    """N = 2^ceil(log2 n)."""
    return 1 << max(0, (int(n) - 1).bit_length())


def _words(count: int, c1: int, seed: int) -> np.ndarray:
    blocks = (count + 3) // 4
    ctr = np.zeros((blocks, 4), dtype=np.uint32)
    ctr[:, 0] = np.arange(blocks, dtype=np.uint32)
    ctr[:, 1] = np.uint32(c1)
    ctr[:, 2] = np.uint32(STREAM_SRHT)
    key = (int(seed) & 0xFFFFFFFF, (int(seed) >> 32) & 0xFFFFFFFF)
    return philox.philox4x32_10(ctr, key).reshape(-1)[:count]


def signs(n: int, seed: int) -> np.ndarray:
    """d_0 .. d_{n-1} in {+1, -1} (float64)."""
    w = _words(n, 0, seed)
    return np.where((w & 1) == 1, -1.0, 1.0)


def subset(N: int, l: int, seed: int) -> np.ndarray:
    """s_0 .. s_{l-1}: the first l picks of the seeded Fisher-Yates shuffle of 0 .. N-1."""
    if not 0 <= l <= N:
        raise ValueError("need 0 <= l <= N")
    u = _words(l, 1, seed).astype(np.uint64)
    perm = np.arange(N, dtype=np.int64)
    for j in range(l):
        r = j + int((int(u[j]) * (N - j)) >> 32)
        perm[j], perm[r] = perm[r], perm[j]
    return perm[:l].copy()


def hadamard(N: int) -> np.ndarray:
    """Sylvester-Hadamard matrix H_N(i, k) = (-1)^popcount(i & k), written from its definition."""
    i = np.arange(N, dtype=np.int64)
    bits = np.bitwise_and(i[:, None], i[None, :])
    par = np.zeros_like(bits)
    while np.any(bits):
        par ^= bits & 1
        bits >>= 1
    return np.where(par == 1, -1.0, 1.0)


def omega(n: int, l: int, seed: int) -> np.ndarray:
    """The n x l test matrix Omega = (D H_N S / sqrt(N))[:n, :], formed explicitly (small n only)."""
    N = padded_size(n)
    d = signs(n, seed)
    s = subset(N, l, seed)
    H = hadamard(N)
    return d[:, None] * H[:n][:, s] / math.sqrt(N)


def sketch(A: np.ndarray, l: int, seed: int) -> np.ndarray:
    """Y = A Omega, by the definition (explicit Omega; a matrix product)."""
    A = np.asarray(A, dtype=np.float64)
    return A @ omega(A.shape[1], l, seed)


def fwht(X: np.ndarray) -> np.ndarray:
    """H_N X for an N x c array X (N a power of two), by butterflies over the bits of the index: at bit h
    the pair (i, i + 2^h), i without bit h, becomes (x_i + x_{i+2^h}, x_i - x_{i+2^h})."""
    Y = np.array(X, dtype=np.float64, copy=True)
    N = Y.shape[0]
    h = 1
    while h < N:
        for start in range(0, N, 2 * h):
            a = Y[start:start + h].copy()
            b = Y[start + h:start + 2 * h].copy()
            Y[start:start + h] = a + b
            Y[start + h:start + 2 * h] = a - b
        h *= 2
    return Y


def sketch_rows(A: np.ndarray, l: int, seed: int) -> np.ndarray:
    """Y = A Omega computed row by row as (H_N (d .* a_r))(S) / sqrt(N), for shapes where the explicit
    Omega would not fit; the same quantity as ``sketch``."""
    A = np.asarray(A, dtype=np.float64)
    m, n = A.shape
    N = padded_size(n)
    X = np.zeros((N, m))
    X[:n] = (A * signs(n, seed)).T
    return fwht(X)[subset(N, l, seed)].T / math.sqrt(N)


def rsvd_srht(A: np.ndarray, k: int, p: int, q: int, seed: int):
    """Figure 5 with the test matrix of Section 6 (l = k + p): Q = orth(A Omega),
    q times { W = orth(A^T Q); Q = orth(A W) }, then Stage B.  Rank-(k+p)
    result (truncate with ``.truncate(k)``)."""
    A = np.asarray(A, dtype=np.float64)
    Y = sketch(A, k + p, seed) if padded_size(A.shape[1]) <= 4096 else sketch_rows(A, k + p, seed)
    Q = orth(Y)
    for _ in range(q):
        W = orth(A.T @ Q)
        Q = orth(A @ W)
    return stage_b(A, Q)
