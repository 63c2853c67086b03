"""Per-kernel parity of the HIP building blocks (include/rsvd_kernels.h)
against CPU references.

Products on small-integer data are exact in every precision (all partial sums
stay below 2^24), so those comparisons are bit for bit.
"""
import ctypes

import numpy as np
import pytest

from tests.gpu_helpers import device

pytestmark = pytest.mark.gpu


def _lib():
    from paper_1607_01649_amd import _lib
    return _lib.lib()


def _t(x, dt):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).to(device(), dt)


def _p(t):
    return ctypes.c_void_p(t.data_ptr())


PREC = {"f64": 0, "f32": 1, "f32acc64": 10}


@pytest.mark.parametrize("prec", ["f64", "f32", "f32acc64"])
@pytest.mark.parametrize("rows,K,ncols,lda_pad", [(128, 64, 16, 0), (300, 517, 30, 0), (77, 1000, 110, 4),
                                                  (1000, 129, 128, 0), (33, 70, 7, 1), (513, 2048, 200, 0)])
def test_product_nn_is_exact_on_integers(prec, rows, K, ncols, lda_pad):
    import torch
    rng = np.random.default_rng(rows + K)
    A = rng.integers(-3, 4, size=(rows, K + lda_pad)).astype(np.float64)
    X = rng.integers(-3, 4, size=(K, ncols)).astype(np.float64)
    ref = A[:, :K] @ X
    tin = torch.float64 if prec == "f64" else torch.float32
    tout = torch.float32 if prec == "f32" else torch.float64
    dA = _t(A, tin)
    ldx = K + 5
    Xp = np.zeros((ncols, ldx))
    Xp[:, :K] = X.T
    dX = _t(Xp, tin)
    ldo = rows + 3
    out = torch.full((ncols, ldo), -7.0, dtype=tout, device=device())
    st = _lib().rsvd_k_product_nn(PREC[prec], rows, K, _p(dA), K + lda_pad, _p(dX), ldx, ncols, _p(out), ldo, None)
    assert st == 0
    got = out.cpu().numpy().astype(np.float64)
    assert np.array_equal(got[:, :rows], ref.T)
    assert np.all(got[:, rows:] == -7.0)     # nothing written past the panel rows


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("K,nc", [(64, 16), (777, 110), (1000, 128), (300, 129), (2049, 300), (5000, 520),
                                  (100, 1), (130, 17), (64, 1024)])
def test_gram_is_exact_on_integers(prec, K, nc):
    """G = Y^T Y through rsvd_k_gram (FP64 accumulation on the FP64 MFMA, upper tile pairs mirrored): exact on
    small integers, both triangles, rows of the panel past K ignored (filled with garbage), nothing written past
    nc rows of G."""
    import torch
    rng = np.random.default_rng(K * 7 + nc)
    Y = rng.integers(-3, 4, size=(K, nc)).astype(np.float64)
    ref = Y.T @ Y
    ldy = (K + 63) // 64 * 64 + 64
    Yp = np.full((nc, ldy), 5.0)          # rows K .. ldy-1 of every column: garbage the kernel must not read in
    Yp[:, :K] = Y.T
    dY = _t(Yp, torch.float64 if prec == "f64" else torch.float32)
    ldg = nc + 3
    G = torch.full((nc, ldg), -7.0, dtype=torch.float64, device=device())
    assert _lib().rsvd_k_gram(PREC[prec], K, nc, _p(dY), ldy, _p(G), ldg, None) == 0
    got = G.cpu().numpy()
    assert np.array_equal(got[:, :nc], ref)
    assert np.all(got[:, nc:] == -7.0)


def test_gram_rejects_bad_arguments():
    import torch
    dY = torch.zeros(64 * 10, dtype=torch.float32, device=device())
    G = torch.zeros(100, dtype=torch.float64, device=device())
    assert _lib().rsvd_k_gram(PREC["f32"], 64, 10, _p(dY), 60, _p(G), 10, None) != 0     # ldy not a multiple of 64
    assert _lib().rsvd_k_gram(PREC["f32"], 65, 1, _p(dY), 64, _p(G), 10, None) != 0     # ldy < K
    assert _lib().rsvd_k_gram(PREC["f32acc64"], 64, 10, _p(dY), 64, _p(G), 10, None) != 0
    assert _lib().rsvd_k_gram(PREC["f32"], 64, 10, _p(dY), 64, _p(G), 9, None) != 0     # ldg < nc


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("K,N,ncols,rowmajor", [(64, 256, 16, 0), (110, 3001, 110, 0), (128, 700, 128, 0),
                                                (517, 300, 30, 0), (1000, 77, 110, 1),
                                                (30, 1000, 30, 0), (129, 513, 200, 1), (2048, 260, 9, 0),
                                                (110, 3001, 100, 1), (128, 700, 128, 1), (7, 50, 5, 1)])
def test_product_tn_is_exact_on_integers(prec, K, N, ncols, rowmajor):
    import torch
    rng = np.random.default_rng(K * 3 + N)
    A = rng.integers(-3, 4, size=(K, N)).astype(np.float64)
    P = rng.integers(-3, 4, size=(K, ncols)).astype(np.float64)
    ref = A.T @ P
    tdt = torch.float64 if prec == "f64" else torch.float32
    dA = _t(A, tdt)
    ldp = K + 2
    Pp = np.zeros((ncols, ldp))
    Pp[:, :K] = P.T
    dP = _t(Pp, tdt)
    if rowmajor:
        ldo = ncols + 3
        out = torch.full((N, ldo), -7.0, dtype=tdt, device=device())
    else:
        ldo = N + 3
        out = torch.full((ncols, ldo), -7.0, dtype=tdt, device=device())
    st = _lib().rsvd_k_product_tn(PREC[prec], K, N, _p(dA), N, _p(dP), ldp, ncols, _p(out), ldo, rowmajor, None)
    assert st == 0
    got = out.cpu().numpy().astype(np.float64)
    if rowmajor:
        assert np.array_equal(got[:, :ncols], ref)
        assert np.all(got[:, ncols:] == -7.0)
    else:
        assert np.array_equal(got[:, :N], ref.T)
        assert np.all(got[:, N:] == -7.0)


def _scratch(l):
    """Device scratch for the kernel-level Cholesky / small SVD at size l."""
    import ctypes
    import torch
    nbytes = ctypes.c_size_t(0)
    assert _lib().rsvd_k_scratch_bytes(l, ctypes.byref(nbytes)) == 0
    return torch.empty(max(nbytes.value, 8), dtype=torch.uint8, device=device())


@pytest.mark.parametrize("l", [1, 5, 16, 30, 110, 128, 129, 200, 520, 1000])
def test_cholesky_and_inverse(l):
    """l <= 128: one workgroup; larger l: the blocked multi-workgroup form
    (64-wide blocks, ragged last block)."""
    import torch
    scr = _scratch(l)
    rng = np.random.default_rng(l)
    Y = rng.standard_normal((3 * l + 5, l)) @ np.diag(np.logspace(0, -3, l))
    G = Y.T @ Y
    LP = (l + 15) // 16 * 16
    dG = _t(G.T, torch.float64)                 # column-major
    Rinv = torch.zeros(LP * LP, dtype=torch.float64, device=device())
    R = torch.zeros(LP * LP, dtype=torch.float64, device=device())
    flags = torch.zeros(4, dtype=torch.int32, device=device())
    st = _lib().rsvd_k_cholesky(l, _p(dG), l, 0.0, _p(Rinv), _p(R), _p(flags), _p(scr), None)
    assert st == 0
    R = R.cpu().numpy().reshape(LP, LP)
    Ri = Rinv.cpu().numpy().reshape(LP, LP).T     # Ri[k, c] = R^-1(k, c)
    assert flags.cpu().numpy()[:2].tolist() == [0, 0]
    Rl = R[:l, :l]
    assert np.allclose(np.tril(Rl, -1), 0) and np.all(np.diag(Rl) > 0)
    ref = np.linalg.cholesky(G).T
    assert np.allclose(Rl, ref, rtol=1e-10, atol=1e-12 * np.abs(ref).max())
    assert np.allclose(Ri[:l, :l] @ Rl, np.eye(l), atol=1e-9)
    assert np.array_equal(R[l:, l:], np.eye(LP - l)) and np.array_equal(Ri[l:, l:], np.eye(LP - l))


def test_cholesky_drops_dependent_columns():
    import torch
    rng = np.random.default_rng(3)
    Y = rng.standard_normal((50, 6))
    Y[:, 3] = Y[:, 0] - 2 * Y[:, 1]          # exactly dependent column
    G = Y.T @ Y
    dG = _t(G.T, torch.float64)
    Rinv = torch.zeros(256, dtype=torch.float64, device=device())
    R = torch.zeros(256, dtype=torch.float64, device=device())
    flags = torch.zeros(4, dtype=torch.int32, device=device())
    # the eliminated pivot of the dependent column is rounding noise, ~u * G_jj
    assert _lib().rsvd_k_cholesky(6, _p(dG), 6, 1e-10, _p(Rinv), _p(R), _p(flags), None, None) == 0
    assert flags.cpu().numpy()[1] == 1
    Ri = Rinv.cpu().numpy().reshape(16, 16).T[:6, :6]
    Q = Y @ Ri
    assert np.allclose(Q[:, 3], 0)
    keep = [0, 1, 2, 4, 5]
    assert np.allclose(Q[:, keep].T @ Q[:, keep], np.eye(5), atol=1e-10)


def test_blocked_cholesky_drops_dependent_columns():
    """l = 200 (64-wide diagonal blocks, ragged last block): exactly dependent columns in the first, an inner
    and the last diagonal block, and one whose dependence spans two blocks, are dropped; the rest of Q is
    orthonormal."""
    import torch
    l = 200
    rng = np.random.default_rng(5)
    Y = rng.standard_normal((700, l))
    dep = {5: (0, 3), 70: (64, 66), 100: (10, 90), 199: (130, 198)}
    for j, (a, b) in dep.items():
        Y[:, j] = Y[:, a] - 0.5 * Y[:, b]
    G = Y.T @ Y
    LP = (l + 15) // 16 * 16
    scr = _scratch(l)
    dG = _t(G.T, torch.float64)
    Rinv = torch.zeros(LP * LP, dtype=torch.float64, device=device())
    R = torch.zeros(LP * LP, dtype=torch.float64, device=device())
    flags = torch.zeros(4, dtype=torch.int32, device=device())
    assert _lib().rsvd_k_cholesky(l, _p(dG), l, 1e-10, _p(Rinv), _p(R), _p(flags), _p(scr), None) == 0
    assert flags.cpu().numpy()[:2].tolist() == [0, len(dep)]
    Ri = Rinv.cpu().numpy().reshape(LP, LP).T[:l, :l]
    Q = Y @ Ri
    drop = sorted(dep)
    keep = [j for j in range(l) if j not in dep]
    assert np.abs(Q[:, drop]).max() <= 1e-12
    assert np.abs(Q[:, keep].T @ Q[:, keep] - np.eye(len(keep))).max() <= 1e-8


@pytest.mark.parametrize("l", [1, 2, 7, 30, 110, 128, 131, 300, 520])
def test_small_svd_matches_lapack(l):
    """R is the triangular factor of a matrix with singular values
    logspace(0, -6, l), so sigma(R^T) is known; LAPACK's SVD is the reference
    for the vectors (absolute accuracy ~ u * sigma_1).  l > 128 runs the block
    one-sided Jacobi over many workgroups."""
    import torch
    scr = _scratch(l)
    from workloads import gen
    s0 = np.logspace(0, -6, l)
    M = (gen.orthonormal_factor(l + 7, l, 100 + l, 1) * s0) @ gen.orthonormal_factor(l, l, 100 + l, 2).T
    R = np.linalg.qr(M, mode="r")
    LP = (l + 15) // 16 * 16
    Rp = np.eye(LP)
    Rp[:l, :l] = R
    dR = _t(Rp, torch.float64)
    sig = torch.zeros(LP, dtype=torch.float64, device=device())
    Uh = torch.zeros(LP * LP, dtype=torch.float64, device=device())
    flags = torch.zeros(4, dtype=torch.int32, device=device())
    assert _lib().rsvd_k_small_svd(l, _p(dR), _p(sig), _p(Uh), _p(flags), _p(scr), None) == 0
    s = sig.cpu().numpy()
    Uh = Uh.cpu().numpy().reshape(LP, LP).T[:l, :l]     # column j of U_hat
    assert np.all(np.abs(s[:l] - s0) <= 1e-13 + 1e-11 * s0)
    assert np.all(s[l:] == 0)
    X = R.T
    W = Uh.T @ X
    # the stopping test leaves |x_p . x_q| <= l u ||x_p|| ||x_q||: bounds grow with l
    assert np.linalg.norm(W @ W.T - np.diag(s[:l] ** 2)) <= max(1e-14 * l, 1e-16 * l * l)
    assert np.linalg.norm(Uh.T @ Uh - np.eye(l)) <= max(1e-12, 1e-15 * l * l)
    ref_u, ref_s, _ = np.linalg.svd(X)
    for j in range(l):
        i = np.argmax(np.abs(Uh[:, j]))
        assert Uh[i, j] > 0
        sgn = np.sign(ref_u[np.argmax(np.abs(ref_u[:, j])), j])
        gap = min([abs(s0[j] - s0[i2]) for i2 in range(l) if i2 != j] + [1.0])
        assert np.linalg.norm(Uh[:, j] - sgn * ref_u[:, j]) <= 1e-13 / gap
    assert flags.cpu().numpy()[2] == 0


@pytest.mark.parametrize("l,r", [(100, 60), (150, 100), (200, 120), (700, 500)])
def test_small_svd_of_a_dense_rank_deficient_matrix(l, r):
    """X = M^T M with M of rank r < l (dense columns; l - r singular values at rounding level): the one-sided
    Jacobi converges, columns whose norm falls to tol ||X||_F or below (tol = l u) come out as sigma = 0 with
    a zero U_hat column, and the others are orthonormal.  l > 128 is the block form (W = 8 at l = 700)."""
    import torch
    g = np.random.default_rng(l + r)
    M = g.standard_normal((l + 50, r)) @ g.standard_normal((r, l))
    X = M.T @ M
    LP = (l + 15) // 16 * 16
    Rp = np.zeros((LP, LP))
    Rp[:l, :l] = X.T                                      # row p of R = column p of X
    scr = _scratch(l)
    dR = _t(Rp, torch.float64)
    sig = torch.zeros(LP, dtype=torch.float64, device=device())
    Uh = torch.zeros(LP * LP, dtype=torch.float64, device=device())
    flags = torch.zeros(4, dtype=torch.int32, device=device())
    assert _lib().rsvd_k_small_svd(l, _p(dR), _p(sig), _p(Uh), _p(flags), _p(scr), None) == 0
    f = flags.cpu().numpy()
    s = sig.cpu().numpy()[:l]
    U = Uh.cpu().numpy().reshape(LP, LP).T[:l, :l]
    ref = np.linalg.svd(X, compute_uv=False)
    nz = s > 0
    print(f"l={l} r={r}: sweeps {f[3]}, nonzero sigma {nz.sum()}", flush=True)
    assert f[0] == 0 and f[2] == 0
    assert np.abs(s - ref).max() <= 1e-12 * ref[0]
    assert nz.sum() >= r and np.all(nz[:nz.sum()])          # zeros only at the end
    assert np.all(s[~nz] == 0) and np.all(U[:, ~nz] == 0)
    assert np.all(ref[~nz] <= l * 2.3e-16 * np.linalg.norm(X))
    Un = U[:, nz]
    assert np.linalg.norm(Un.T @ Un - np.eye(nz.sum())) <= 1e-10
    # U_hat^T X X^T U_hat is diagonal up to the stopping test (|x_p . x_q| <= l u ||x_p|| ||x_q||)
    assert np.linalg.norm((U.T @ X) @ (X.T @ U) - np.diag(s ** 2)) <= 1e-16 * l * l * ref[0] ** 2


def test_convert_bf16_is_bit_exact():
    import torch
    from oracle import quant
    rng = np.random.default_rng(11)
    m, n = 300, 517
    A = (rng.standard_normal((m, n)) * 10).astype(np.float32)
    # exact ties and tiny values
    A[0, :8] = ((np.arange(8, dtype=np.uint32) * 0x10000 + 0x3F808000).view(np.float32))
    A[1, :3] = np.array([1e-40, -3e-39, 1e-45], dtype=np.float32)
    ld16, ldT = 640, 384
    dA = _t(A, torch.float32)
    A16 = torch.full((m, ld16), -1, dtype=torch.int16, device=device())
    A16T = torch.full((n, ldT), -1, dtype=torch.int16, device=device())
    flag = torch.zeros(1, dtype=torch.int32, device=device())
    assert _lib().rsvd_k_convert_bf16(m, n, _p(dA), n, _p(A16), ld16, _p(A16T), ldT, _p(flag), None) == 0
    got = A16.cpu().numpy().view(np.uint16)
    want = quant.bf16_bits(A)
    assert np.array_equal(got[:, :n], want)
    assert np.all(got[:, n:] == 0)
    gt = A16T.cpu().numpy().view(np.uint16)
    assert np.array_equal(gt[:, :m], want.T)
    assert np.all(gt[:, m:] == 0)
    assert int(flag.cpu()[0]) == 0
    A[5, 7] = np.inf
    dA = _t(A, torch.float32)
    assert _lib().rsvd_k_convert_bf16(m, n, _p(dA), n, _p(A16), ld16, _p(A16T), ldT, _p(flag), None) == 0
    assert int(flag.cpu()[0]) == 1


@pytest.mark.parametrize("rows,K,ncols", [(128, 128, 16), (300, 517, 30), (77, 1000, 110), (1000, 129, 128),
                                          (33, 70, 7), (513, 2048, 200)])
def test_product_bf16_is_exact_on_integers(rows, K, ncols):
    import torch
    rng = np.random.default_rng(rows * 7 + K)
    A = rng.integers(-16, 17, size=(rows, K)).astype(np.float32)
    X = rng.integers(-16, 17, size=(K, ncols)).astype(np.float32)
    ref = A.astype(np.float64) @ X.astype(np.float64)
    lda = (K + 127) // 128 * 128
    ldT = (rows + 127) // 128 * 128
    dA = _t(A, torch.float32)
    A16 = torch.zeros((rows, lda), dtype=torch.int16, device=device())
    A16T = torch.zeros((K, ldT), dtype=torch.int16, device=device())
    flag = torch.zeros(1, dtype=torch.int32, device=device())
    assert _lib().rsvd_k_convert_bf16(rows, K, _p(dA), K, _p(A16), lda, _p(A16T), ldT, _p(flag), None) == 0
    ldx = (K + 3) // 4 * 4 + 4
    Xp = np.zeros((ncols, ldx), dtype=np.float32)
    Xp[:, :K] = X.T
    dX = _t(Xp, torch.float32)
    ldo = rows + 3
    out = torch.full((ncols, ldo), -7.0, dtype=torch.float32, device=device())
    assert _lib().rsvd_k_product_bf16(rows, K, _p(A16), lda, _p(dX), ldx, ncols, _p(out), ldo,
                                      _p(_lp_scratch("bf16", K, ncols)), None) == 0
    got = out.cpu().numpy().astype(np.float64)
    assert np.array_equal(got[:, :rows], ref.T)
    assert np.all(got[:, rows:] == -7.0)
    # and the transposed copy gives A^T P
    P = rng.integers(-16, 17, size=(rows, 9)).astype(np.float32)
    ldp = ldT
    Pp = np.zeros((9, ldp), dtype=np.float32)
    Pp[:, :rows] = P.T
    dP = _t(Pp, torch.float32)
    out2 = torch.zeros((9, K), dtype=torch.float32, device=device())
    assert _lib().rsvd_k_product_bf16(K, rows, _p(A16T), ldT, _p(dP), ldp, 9, _p(out2), K,
                                      _p(_lp_scratch("bf16", rows, 9)), None) == 0
    assert np.array_equal(out2.cpu().numpy().astype(np.float64), (A.astype(np.float64).T @ P).T)


def _lp_scratch(dtype, K, ncols):
    """Device scratch for the thin operand of a low-precision product."""
    import torch
    nbytes = ctypes.c_size_t(0)
    code = {"bf16": 2, "fp8": 3}[dtype]
    assert _lib().rsvd_k_lp_scratch_bytes(code, K, ncols, ctypes.byref(nbytes)) == 0
    buf = torch.empty(nbytes.value + 256, dtype=torch.uint8, device=device())
    off = (-buf.data_ptr()) % 256
    return buf[off:off + nbytes.value]


def _fp8_convert(A, torch):
    m, n = A.shape
    ld8, ldT = (n + 127) // 128 * 128, (m + 127) // 128 * 128
    dA = _t(A, torch.float32)
    A8 = torch.full((m, ld8), 0x55, dtype=torch.uint8, device=device())
    A8T = torch.full((n, ldT), 0x55, dtype=torch.uint8, device=device())
    sc = torch.zeros((ldT // 128) * (ld8 // 128), dtype=torch.float32, device=device())
    flag = torch.zeros(1, dtype=torch.int32, device=device())
    assert _lib().rsvd_k_convert_fp8(m, n, _p(dA), n, _p(A8), ld8, _p(A8T), ldT, _p(sc), _p(flag), None) == 0
    return A8, A8T, sc, flag, ld8, ldT


def test_convert_fp8_is_bit_exact():
    """E4M3 codes of both copies and the power-of-two tile scales equal the
    oracle's (ragged tiles, tiles of very different magnitude, exact ties,
    saturation-free by construction, values that round to zero)."""
    import torch
    from oracle import quant
    rng = np.random.default_rng(12)
    m, n = 300, 517
    A = (rng.standard_normal((m, n)) * np.exp(rng.uniform(-8, 8, (m, 1)))).astype(np.float32)
    A[:128, :128] *= np.float32(1e-30)           # a tile far below the others
    A[128:256, 128:256] *= np.float32(1e-40)     # a tile (mostly subnormal) at the lower limit of the E8M0 scale
    A[200, :8] = np.array([1.0, 1.0625, 1.1875, 3.0, 2 ** -10, -2 ** -9, 0.0, -0.0], dtype=np.float32)
    A8, A8T, sc, flag, ld8, ldT = _fp8_convert(A, torch)
    codes, ex, _ = quant.fp8_blocks_matrix(A)
    got = A8.cpu().numpy()
    assert np.array_equal(got[:, :n], codes)
    assert np.all(got[:, n:] == 0)
    gt = A8T.cpu().numpy()
    assert np.array_equal(gt[:, :m], codes.T)
    assert np.all(gt[:, m:] == 0)
    want_sc = np.zeros((ldT // 128, ld8 // 128))
    want_sc[:ex.shape[0], :ex.shape[1]] = 2.0 ** ex
    assert np.array_equal(sc.cpu().numpy().reshape(want_sc.shape)[:ex.shape[0], :ex.shape[1]],
                          want_sc[:ex.shape[0], :ex.shape[1]])
    assert int(flag.cpu()[0]) == 0
    A[5, 7] = np.nan
    _, _, _, flag, _, _ = _fp8_convert(A, torch)
    assert int(flag.cpu()[0]) == 1


@pytest.mark.parametrize("rows,K,ncols", [(128, 128, 16), (300, 517, 30), (77, 1000, 110), (1000, 129, 128),
                                          (33, 70, 7), (513, 2048, 200), (300, 700, 520)])
def test_product_fp8_is_exact_on_integers(rows, K, ncols):
    """Integers of magnitude <= 16 stay exact under the block scales and the
    FP32 sums stay below 2^24: A X and (through the transposed copy) A^T P are
    bit-exact."""
    import torch
    rng = np.random.default_rng(rows * 11 + K)
    A = rng.integers(-16, 17, size=(rows, K)).astype(np.float32)
    X = rng.integers(-16, 17, size=(K, ncols)).astype(np.float32)
    A8, A8T, sc, flag, lda, ldT = _fp8_convert(A, torch)
    ntc = lda // 128
    ldx = (K + 3) // 4 * 4 + 4
    Xp = np.zeros((ncols, ldx), dtype=np.float32)
    Xp[:, :K] = X.T
    ldo = rows + 3
    out = torch.full((ncols, ldo), -7.0, dtype=torch.float32, device=device())
    assert _lib().rsvd_k_product_fp8(rows, K, _p(A8), lda, _p(sc), ntc, 1, _p(_t(Xp, torch.float32)), ldx, ncols,
                                     _p(out), ldo, _p(_lp_scratch("fp8", K, ncols)), None) == 0
    got = out.cpu().numpy().astype(np.float64)
    assert np.array_equal(got[:, :rows], (A.astype(np.float64) @ X.astype(np.float64)).T)
    assert np.all(got[:, rows:] == -7.0)
    P = rng.integers(-16, 17, size=(rows, 9)).astype(np.float32)
    Pp = np.zeros((9, ldT), dtype=np.float32)
    Pp[:, :rows] = P.T
    out2 = torch.zeros((9, K), dtype=torch.float32, device=device())
    assert _lib().rsvd_k_product_fp8(K, rows, _p(A8T), ldT, _p(sc), 1, ntc, _p(_t(Pp, torch.float32)), ldT, 9,
                                     _p(out2), K, _p(_lp_scratch("fp8", rows, 9)), None) == 0
    assert np.array_equal(out2.cpu().numpy().astype(np.float64), (A.astype(np.float64).T @ P).T)


def test_product_fp8_matches_the_dequantised_operands():
    """Random data: the product equals the FP64 product of the oracle's
    dequantised operands within FP32 accumulation error."""
    import torch
    from oracle import quant
    rng = np.random.default_rng(3)
    rows, K, ncols = 700, 1300, 40
    A = (rng.standard_normal((rows, K)) * np.exp(rng.uniform(-3, 3, (1, K)))).astype(np.float32)
    X = rng.standard_normal((K, ncols)).astype(np.float32)
    A8, A8T, sc, flag, lda, ldT = _fp8_convert(A, torch)
    ldx = (K + 3) // 4 * 4
    Xp = np.zeros((ncols, ldx), dtype=np.float32)
    Xp[:, :K] = X.T
    out = torch.zeros((ncols, rows), dtype=torch.float32, device=device())
    assert _lib().rsvd_k_product_fp8(rows, K, _p(A8), lda, _p(sc), lda // 128, 1, _p(_t(Xp, torch.float32)), ldx,
                                     ncols, _p(out), rows, _p(_lp_scratch("fp8", K, ncols)), None) == 0
    Aq = quant.fp8_blocks_matrix(A)[2]
    Xq = quant.fp8_round_thin(X)
    ref = Aq @ Xq
    bound = 2 * K * 2.0 ** -24 * (np.abs(Aq) @ np.abs(Xq))
    assert np.all(np.abs(out.cpu().numpy().T - ref) <= bound)

