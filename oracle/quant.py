"""Rounding to the low-precision operand formats, and the quantisation-aware
form of the randomized SVD.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper's algorithms are stated in exact arithmetic.  When the products
with A take their operands in a narrow format, the computed factors are those
of the rounded operands; this module rounds the operands exactly as the
format defines (bfloat16: the top 16 bits of the binary32 encoding, round to
nearest, ties to even) and then runs Figure 5 in float64 on them, so that the
remaining difference from a GPU run is arithmetic (accumulation) error only.
The error of the format itself is measured against the plain oracle.
"""
from __future__ import annotations

import numpy as np

from . import rsvd as _r


def bf16_round(x) -> np.ndarray:
    """Round to bfloat16 (from the binary32 value of x), ties to even; NaN
    stays NaN.  Returned as float64 (exactly representable)."""
    x32 = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    u = x32.view(np.uint32).astype(np.uint64)
    nan = (u & 0x7FFFFFFF) > 0x7F800000
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) & 0xFFFF
    r = np.where(nan, (u >> 16) | 0x40, r)
    return (r.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def bf16_bits(x) -> np.ndarray:
    """The 16-bit bfloat16 codes of bf16_round(x)."""
    return (bf16_round(x).astype(np.float32).view(np.uint32) >> 16).astype(np.uint16)


ROUNDERS = {"f32": lambda x: np.asarray(x, dtype=np.float32).astype(np.float64), "bf16": bf16_round}


def rsvd_quantized(A, G, q, sketch: str = "bf16", proj: str = "bf16") -> "_r.RSVDResult":
    """Figure 5 with every operand of a product with A rounded to its format:
    A and the thin operand (Omega, W, Q, first rounded to binary32 as the GPU
    keeps them) of A*X, A^T*X in the `sketch` format and of the projection
    B = Q^T A in the `proj` format; orth and the small SVD exact (float64)."""
    rs, rp = ROUNDERS[sketch], ROUNDERS[proj]
    A = np.asarray(A, dtype=np.float64)
    As, Ap = rs(A), rp(A)

    def thin(X, r):
        return r(np.asarray(X, dtype=np.float32))
    Q = _r.orth(As @ thin(G, rs))
    for _ in range(q):
        W = _r.orth(As.T @ thin(Q, rs))
        Q = _r.orth(As @ thin(W, rs))
    B = thin(Q, rp).T @ Ap
    uh, d, v = _r.svd_small(B)
    return _r.RSVDResult(Q @ uh, d, v, Q, B)
