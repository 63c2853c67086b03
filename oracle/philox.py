"""Philox4x32-10 and Box-Muller Gaussians, written from the published
definition (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy as
1, 2, 3", SC'11, Section 4 / the Philox-4x32 round function).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper asks for a Gaussian test matrix (Section 4, Figure 1 step 1; Figure
5 step 1) without naming a generator.  The reading used throughout: entry
(i, j) of a Gaussian matrix drawn from ``(seed, stream)`` is a function of
(seed, stream, i, j) only, so column prefixes are stable when more columns
are drawn later (the adaptive finders of Sections 12-13 draw further
Gaussian vectors one block at a time).

Mapping (shared definition, implemented independently on each side):
  key     = (seed mod 2^32, seed div 2^32)
  counter = (i div 2, j, stream, 0)
  (x0, x1, x2, x3) = Philox4x32-10(counter, key)
  u1 = ((x0 * 2^32 + x1) div 2^11 + 1/2) * 2^-53        (in (0, 1))
  u2 = ((x2 * 2^32 + x3) div 2^11 + 1/2) * 2^-53
  rad = sqrt(-2 ln u1), theta = 2 pi u2
  entry (i, j) = rad * cos(theta) if i is even else rad * sin(theta)
"""
from __future__ import annotations

import numpy as np

_M0 = np.uint64(0xD2511F53)
_M1 = np.uint64(0xCD9E8D57)
_W0 = 0x9E3779B9
_W1 = 0xBB67AE85
_MASK32 = np.uint64(0xFFFFFFFF)


def philox4x32_10(ctr: np.ndarray, key) -> np.ndarray:
    """Philox4x32 with 10 rounds.

    ``ctr``: uint32 array of shape (..., 4); ``key``: two 32-bit integers.
    Returns a uint32 array of the same shape.  One round maps
    (c0, c1, c2, c3) to (hi(M1*c2) ^ c1 ^ k0, lo(M1*c2), hi(M0*c0) ^ c3 ^ k1,
    lo(M0*c0)); the key is bumped by the Weyl constants between rounds.
    """
    c = np.asarray(ctr, dtype=np.uint32).astype(np.uint64)
    c0, c1, c2, c3 = c[..., 0], c[..., 1], c[..., 2], c[..., 3]
    k0, k1 = int(key[0]) & 0xFFFFFFFF, int(key[1]) & 0xFFFFFFFF
    for rnd in range(10):
        if rnd > 0:
            k0 = (k0 + _W0) & 0xFFFFFFFF
            k1 = (k1 + _W1) & 0xFFFFFFFF
        p0 = _M0 * c0
        p1 = _M1 * c2
        hi0, lo0 = p0 >> np.uint64(32), p0 & _MASK32
        hi1, lo1 = p1 >> np.uint64(32), p1 & _MASK32
        c0, c1, c2, c3 = (hi1 ^ c1 ^ np.uint64(k0)), lo1, (hi0 ^ c3 ^ np.uint64(k1)), lo0
    return np.stack([c0, c1, c2, c3], axis=-1).astype(np.uint32)


def _counters(rows: int, col0: int, cols: int, stream: int) -> np.ndarray:
    pairs = (rows + 1) // 2
    i2 = np.arange(pairs, dtype=np.uint32)
    j = np.arange(col0, col0 + cols, dtype=np.uint32)
    ctr = np.zeros((pairs, cols, 4), dtype=np.uint32)
    ctr[..., 0] = i2[:, None]
    ctr[..., 1] = j[None, :]
    ctr[..., 2] = np.uint32(stream)
    return ctr


def gaussian(rows: int, cols: int, seed: int, stream: int, col0: int = 0) -> np.ndarray:
    """rows x cols float64 standard Gaussian matrix, columns col0 .. col0+cols-1
    of the (seed, stream) family, by the mapping in the module docstring."""
    key = (int(seed) & 0xFFFFFFFF, (int(seed) >> 32) & 0xFFFFFFFF)
    x = philox4x32_10(_counters(rows, col0, cols, stream), key).astype(np.uint64)
    v1 = ((x[..., 0] << np.uint64(32)) | x[..., 1]) >> np.uint64(11)
    v2 = ((x[..., 2] << np.uint64(32)) | x[..., 3]) >> np.uint64(11)
    u1 = (v1.astype(np.float64) + 0.5) * 2.0 ** -53
    u2 = (v2.astype(np.float64) + 0.5) * 2.0 ** -53
    rad = np.sqrt(-2.0 * np.log(u1))
    theta = 2.0 * np.pi * u2
    out = np.empty((2 * x.shape[0], cols))
    out[0::2] = rad * np.cos(theta)
    out[1::2] = rad * np.sin(theta)
    return out[:rows]


# Stream identifiers of the method's random draws (same numbers on both sides).
STREAM_OMEGA = 4      # the test matrix Omega and, by prefix extension, fallback blocks
STREAM_PROBE = 5      # the 16-column probe sketch read by the (p, q) selector
STREAM_CERT = 6       # the certificate's Gaussian vectors
