"""Host replays of kernel index arithmetic (no GPU): every index a launch can
form is checked against the extent of the buffer it reads.

The FP8 product reads one E8M0 tile scale per (wave, chunk) at
scale[tile_row * s_row + chunk * s_k].  Waves past the last row work on the
clamped row rows - 1 (never stored) and must take that row's tile, or they read
one tile row past a table sized ceil(rows/128) x ceil(K/128)."""
import itertools

import pytest

LROWS = 256        # rows per workgroup (four waves of 64)
WAVE_ROWS = 64
LKC = 128


def _lp_nb_fp8(ncols):
    nb = (ncols + 15) // 16
    groups = (nb + 11) // 12
    nb = (nb + groups - 1) // groups
    return (nb + 1) & ~1


def _fp8_scale_indices(rows, K, ncols, s_row, s_k, splits):
    """Every scale index the FP8 product's grid forms (mirror of the kernel's
    workgroup -> (row block, column group) map and its chunk clamping)."""
    nb = _lp_nb_fp8(ncols)
    cpad = -(-ncols // (16 * nb)) * 16 * nb
    groups = cpad // (nb * 16)
    rblocks = -(-rows // LROWS)
    slots = -(-rblocks // 8) * groups
    kchunk = max(LKC, (-(-K // splits) + LKC - 1) // LKC * LKC)
    used = -(-K // kchunk)
    out = set()
    for bx, split in itertools.product(range(slots * 8), range(used)):
        slot, xcd = bx >> 3, bx & 7
        rb = (slot // groups) * 8 + xcd
        if rb >= rblocks:
            continue
        kbeg = split * kchunk
        kend = min(K, kbeg + kchunk)
        nck = -(-(kend - kbeg) // LKC)
        for wave in range(4):
            rbase = rb * LROWS + wave * WAVE_ROWS
            trow = min(rbase, rows - 1) // 128
            for i in range(nck):
                k0 = kbeg + min(i, nck - 1) * LKC
                out.add(trow * s_row + (k0 // LKC) * s_k)
    return out


@pytest.mark.parametrize("rows_mod", [1, 44, 128, 129, 255, 0])
@pytest.mark.parametrize("orient", ["A", "AT"])
@pytest.mark.parametrize("splits", [1, 3])
def test_fp8_scale_index_stays_inside_the_table(rows_mod, orient, splits):
    rows = 4 * 256 + rows_mod if rows_mod else 4 * 256
    K = 517
    ntr, ntk = -(-rows // 128), -(-K // 128)
    # A orientation: table rows = row tiles, s_row = tiles per row; A^T: s_row = 1, s_k = row tiles of A
    s_row, s_k = (ntk, 1) if orient == "A" else (1, ntr)
    size = ntr * ntk
    idx = _fp8_scale_indices(rows, K, 520, s_row, s_k, splits)
    assert min(idx) >= 0 and max(idx) < size, (rows, max(idx), size)
    # every tile of the table is read by some wave
    assert len(idx) == size


def test_the_unclamped_row_would_overrun():
    """The check above can fail: with the tile row taken from the wave's first
    row unclamped, rows mod 256 in [1, 128] reads tile row ceil(rows/128)."""
    rows, K = 1024 + 44, 256
    ntr = -(-rows // 128)
    rblocks = -(-rows // LROWS)
    worst = max((rb * LROWS + w * WAVE_ROWS) // 128 for rb in range(rblocks) for w in range(4))
    assert worst >= ntr
