"""Rounding to the low-precision operand formats, and the quantisation-aware
form of the randomized SVD.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper's algorithms are stated in exact arithmetic.  When the products
with A take their operands in a narrow format, the computed factors are those
of the rounded operands; this module rounds the operands exactly as the
format defines and then runs Figure 5 in float64 on them, so that the
remaining difference from a GPU run is arithmetic (accumulation) error only.
The error of the format itself is measured against the plain oracle.

Formats
  bfloat16   the top 16 bits of the binary32 encoding, round to nearest, ties
             to even.
  FP8 E4M3   the OCP 8-bit format with 4 exponent bits (bias 7) and 3
             mantissa bits, no infinities, largest finite value 448; round to
             nearest, ties to even (the even code), saturating at +-448.  Used
             with power-of-two block scales: a block with largest magnitude
             amax gets the scale 2^e, e the least integer with amax <= 448 2^e
             (e = 0 for an all-zero block), and stores round(x / 2^e).  The
             blocks are 128 x 128 tiles of A (one copy serves A X and A^T X)
             and 128-row segments of each column of a thin operand.
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


def _e4m3_table() -> np.ndarray:
    """Values of the codes 0x00 .. 0x7E (non-negative finite E4M3), ascending."""
    vals = []
    for c in range(0x7F):
        e, m = c >> 3, c & 7
        vals.append(m / 8.0 * 2.0 ** -6 if e == 0 else (1.0 + m / 8.0) * 2.0 ** (e - 7))
    return np.array(vals)


E4M3_VALUES = _e4m3_table()
E4M3_MAX = 448.0


def fp8_e4m3_bits(x) -> np.ndarray:
    """E4M3 codes of x (float64 input): nearest value, ties to the even code,
    magnitudes above 448 saturated, NaN -> 0x7F (sign kept)."""
    x = np.asarray(x, dtype=np.float64)
    a = np.abs(x)
    hi = np.clip(np.searchsorted(E4M3_VALUES, a, side="left"), 0, len(E4M3_VALUES) - 1)   # first value >= a
    lo = np.maximum(hi - 1, 0)
    dlo = a - E4M3_VALUES[lo]
    dhi = E4M3_VALUES[hi] - a
    pick_hi = (dhi < dlo) | ((dhi == dlo) & (hi % 2 == 0))
    code = np.where(pick_hi, hi, lo)
    code = np.where(a >= E4M3_MAX, 0x7E, code)
    code = np.where(np.isnan(x), 0x7F, code)
    return (code | np.where(np.signbit(x), 0x80, 0)).astype(np.uint8)


def fp8_e4m3_decode(codes) -> np.ndarray:
    c = np.asarray(codes, dtype=np.int64)
    mag = c & 0x7F
    v = np.where(mag == 0x7F, np.nan, E4M3_VALUES[np.minimum(mag, 0x7E)])
    return np.where(c & 0x80, -v, v)


def fp8_e4m3_round(x) -> np.ndarray:
    return fp8_e4m3_decode(fp8_e4m3_bits(x))


def fp8_scale_exponent(amax) -> np.ndarray:
    """Least e with amax <= 448 2^e (0 where amax == 0), for the binary32
    value of amax, and at least -127 (the smallest E8M0 scale).  With
    amax = f 2^E, f in [0.5, 1), and 448 = 0.875 2^9: e = E - 9 when
    f <= 0.875, else E - 8 (exact, no logarithm)."""
    a = np.asarray(amax, dtype=np.float32).astype(np.float64)
    f, E = np.frexp(a)                   # a = f 2^E, f in [0.5, 1)
    e = np.maximum(np.where(f <= 0.875, E - 9, E - 8), -127)
    return np.where(a > 0, e, 0).astype(np.int64)


def fp8_blocks_matrix(A, tile: int = 128):
    """A (rows x cols) -> (codes, tile exponents, dequantized value) with one
    scale per tile x tile block (binary32 input)."""
    A32 = np.asarray(A, dtype=np.float32).astype(np.float64)
    r, c = A32.shape
    tr, tc = (r + tile - 1) // tile, (c + tile - 1) // tile
    ex = np.zeros((tr, tc), np.int64)
    codes = np.zeros((r, c), np.uint8)
    deq = np.zeros((r, c))
    for i in range(tr):
        for j in range(tc):
            blk = A32[i * tile:(i + 1) * tile, j * tile:(j + 1) * tile]
            e = int(fp8_scale_exponent(np.max(np.abs(blk)) if blk.size else 0.0))
            ex[i, j] = e
            cd = fp8_e4m3_bits(blk * 2.0 ** -e)
            codes[i * tile:(i + 1) * tile, j * tile:(j + 1) * tile] = cd
            deq[i * tile:(i + 1) * tile, j * tile:(j + 1) * tile] = fp8_e4m3_decode(cd) * 2.0 ** e
    return codes, ex, deq


def fp8_round_thin(X, seg: int = 128) -> np.ndarray:
    """Thin operand X (K x c, binary32 values): each column's 128-row segments
    scaled and rounded on their own; returns the dequantized values."""
    X32 = np.asarray(X, dtype=np.float32).astype(np.float64)
    out = np.zeros_like(X32)
    for j in range(X32.shape[1]):
        for k0 in range(0, X32.shape[0], seg):
            s = X32[k0:k0 + seg, j]
            e = int(fp8_scale_exponent(np.max(np.abs(s)) if s.size else 0.0))
            out[k0:k0 + seg, j] = fp8_e4m3_round(s * 2.0 ** -e) * 2.0 ** e
    return out


ROUNDERS = {"f32": lambda x: np.asarray(x, dtype=np.float32).astype(np.float64), "bf16": bf16_round,
            "fp8": fp8_round_thin}
BIG_ROUNDERS = {"f32": ROUNDERS["f32"], "bf16": bf16_round, "fp8": lambda A: fp8_blocks_matrix(A)[2]}


def rsvd_quantized(A, G, q, sketch: str = "bf16", proj: str = "bf16") -> "_r.RSVDResult":
    """Figure 5 with every operand of a product with A rounded to its format:
    A and the thin operand (Omega, W, Q, first rounded to binary32 as the GPU
    keeps them) of A*X, A^T*X in the `sketch` format and of the projection
    B = Q^T A in the `proj` format; orth and the small SVD exact (float64).
    FP8: A with 128 x 128 tile scales, thin operands with 128-row segment
    scales per column (segments counted from row 0 of the contraction)."""
    rs, rp = ROUNDERS[sketch], ROUNDERS[proj]
    A = np.asarray(A, dtype=np.float64)
    As, Ap = BIG_ROUNDERS[sketch](A), BIG_ROUNDERS[proj](A)

    def thin(X, r):
        return r(np.asarray(X, dtype=np.float32))
    Q = _r.orth(As @ thin(G, rs))
    for _ in range(q):
        W = _r.orth(As.T @ thin(Q, rs))
        Q = _r.orth(As @ thin(W, rs))
    B = thin(Q, rp).T @ Ap
    uh, d, v = _r.svd_small(B)
    return _r.RSVDResult(Q @ uh, d, v, Q, B)
