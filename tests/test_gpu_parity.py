"""Parity of the HIP path (through the C ABI) with the float64 CPU oracle.

Tolerances
  FP64 path: singular values relative error <= 1e-10; U and V columns within
             1e-8 (the oracle and the GPU use the same sign rule), which is
             u64 * kappa / gap with a wide margin for these spectra.
  FP32 path: singular values relative error <= 1e-4 against the FP64 oracle;
             rank-k subspaces within sin(theta) <= 50 * sqrt(n) * u32 / relgap,
             relgap = (sigma_k - sigma_{k+1}) / sigma_1 of the oracle's factors
             (a Wedin-type bound with the FP32 rounding of the data as the
             perturbation).
"""
import math

import numpy as np
import pytest

from oracle import philox, rsvd as orc
from workloads import gen

from tests.gpu_helpers import column_errors, device, max_rel_sigma, orth_error, run_factor, subspace_sin

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24


def _kat_rows(golden_dir):
    import os
    rows = []
    for line in open(os.path.join(golden_dir, "philox4x32_10_kat.txt")):
        if line.strip() and not line.startswith("#"):
            rows.append([int(w, 16) for w in line.split()])
    return rows


def test_philox_known_answers_on_device(golden_dir):
    import torch
    from paper_1607_01649_amd import rsvd_philox4x32_10
    dev = device()
    for r in _kat_rows(golden_dir):
        ctr = torch.tensor(np.array(r[0:4], dtype=np.uint32).view(np.int32)[None, :], device=dev)
        out = torch.empty_like(ctr)
        rsvd_philox4x32_10(ctr, r[4], r[5], out)
        got = out.cpu().numpy().view(np.uint32)[0].tolist()
        assert got == r[6:10]
    # a batch of counters against the oracle's integers, bit for bit
    rng = np.random.default_rng(0)
    c = rng.integers(0, 2 ** 32, size=(4096, 4), dtype=np.uint64).astype(np.uint32)
    ctr = torch.tensor(c.view(np.int32), device=dev)
    out = torch.empty_like(ctr)
    rsvd_philox4x32_10(ctr, 0x12345678, 0x9ABCDEF0, out)
    assert np.array_equal(out.cpu().numpy().view(np.uint32), philox.philox4x32_10(c, (0x12345678, 0x9ABCDEF0)))


@pytest.mark.parametrize("rows,cols,col0", [(1001, 7, 0), (64, 33, 5), (2, 1, 1000)])
def test_gaussian_matches_the_oracle_generator(rows, cols, col0):
    import torch
    from paper_1607_01649_amd import rsvd_gaussian
    dev = device()
    ref = philox.gaussian(rows, cols, 987654321123, 4, col0=col0)
    out = torch.empty(rows, cols, dtype=torch.float64, device=dev)
    rsvd_gaussian(987654321123, 4, out, col0=col0)
    got = out.cpu().numpy()
    # same integers; log/cos/sin of the two math libraries agree to a few ulp
    assert np.max(np.abs(got - ref) / np.maximum(1.0, np.abs(ref))) < 1e-14
    out32 = torch.empty(rows, cols, dtype=torch.float32, device=dev)
    rsvd_gaussian(987654321123, 4, out32, col0=col0)
    assert np.max(np.abs(out32.cpu().numpy() - ref.astype(np.float32))) <= 2 * U32 * np.max(np.abs(ref))


F64_CASES = [
    # m, n, rank, alpha, k, p, q
    (600, 500, 120, 2.0, 20, 10, 1),
    (517, 389, 100, 1.0, 7, 6, 0),     # ragged tails everywhere, q = 0
    (300, 300, 300, 1.0, 290, 10, 2),  # k + p = min(m, n)
    (128, 96, 60, 1.5, 16, 0, 1),      # p = 0
    (1000, 64, 64, 1.0, 40, 24, 1),    # l = n
    (70, 900, 70, 1.0, 20, 15, 2),     # wide A
]


@pytest.mark.parametrize("m,n,rank,alpha,k,p,q", F64_CASES)
def test_factor_f64_matches_the_oracle_given_omega(m, n, rank, alpha, k, p, q):
    sigma = gen.spectrum("poly", rank, alpha=alpha)
    A = gen.low_rank_matrix(m, n, sigma, 1e-8, seed=m * 7 + n)
    G = gen.gaussian_matrix(n, k + p, seed=m + n)
    ref = orc.rsvd(A, G, q).truncate(k)
    U, S, V, info = run_factor(A, k, p, q, "f64", omega=G)
    assert info.status == 0 and info.rank_out == k
    assert max_rel_sigma(S, ref.D, k) <= 1e-10
    gaps = np.abs(np.diff(ref.D))
    good = [j for j in range(k) if (j == 0 or gaps[j - 1] > 1e-6 * ref.D[0]) and (j >= len(gaps) or gaps[j] > 1e-6 * ref.D[0])]
    assert column_errors(U[:, good], ref.U[:, good]) <= 1e-8
    assert column_errors(V[:, good], ref.V[:, good]) <= 1e-8


def test_factor_f64_plain_2000_from_seed():
    """The 2000 x 2000 float64 workload (sigma_j = j^-2 over 200 modes, noise
    1e-8, k=20, p=10, q=1) with Omega drawn on the device from the seed and
    independently by the oracle's own Philox generator."""
    cfg = gen.config("plain_f64_2000")
    A = cfg.matrix(seed=11)
    ref = orc.rsvd_seeded(A, cfg.k, cfg.p, cfg.q, seed=2024).truncate(cfg.k)
    U, S, V, info = run_factor(A, cfg.k, cfg.p, cfg.q, "f64", seed=2024)
    assert max_rel_sigma(S, ref.D, cfg.k) <= 1e-10
    assert column_errors(U, ref.U) <= 1e-8
    assert column_errors(V, ref.V) <= 1e-8
    # the Eckart-Young floor holds for the returned rank-k factors
    err = np.linalg.norm(A - (U * S) @ V.T, 2)
    s = np.linalg.svd(A, compute_uv=False)
    assert err >= s[cfg.k] * (1 - 1e-10)


F32_CASES = [
    # m, n, rank, alpha, k, p, q, lda_pad
    (3000, 1500, 300, 0.5, 20, 10, 2, 0),
    (1237, 901, 200, 1.0, 12, 8, 1, 0),    # n % 4 != 0: unaligned rows, scalar loads
    (2048, 1024, 256, 0.5, 50, 14, 2, 3),  # lda = n + 3
    (777, 2500, 150, 0.8, 30, 10, 1, 0),
    (2000, 1500, 400, 0.5, 180, 20, 1, 0),  # l = 200: blocked Cholesky, triangular apply over two column groups
]


@pytest.mark.parametrize("m,n,rank,alpha,k,p,q,pad", F32_CASES)
def test_factor_f32_matches_the_f64_oracle(m, n, rank, alpha, k, p, q, pad):
    sigma = gen.spectrum("poly", rank, alpha=alpha)
    A64 = gen.low_rank_matrix(m, n, sigma, 1e-3 / math.sqrt(n), seed=m + 3 * n)
    A32 = A64.astype(np.float32)
    G = gen.gaussian_matrix(n, k + p, seed=m * n)
    ref = orc.rsvd(A32.astype(np.float64), G, q)
    refk = ref.truncate(k)
    U, S, V, info = run_factor(A32, k, p, q, "f32", omega=G, lda_pad=pad)
    assert info.status == 0
    assert max_rel_sigma(S, refk.D, k) <= 1e-4
    relgap = (ref.D[k - 1] - ref.D[k]) / ref.D[0]
    tol = 50 * math.sqrt(max(m, n)) * U32 / relgap
    assert subspace_sin(U, refk.U) <= tol
    assert subspace_sin(V, refk.V) <= tol
    assert orth_error(U) <= 1e-5 and orth_error(V) <= 1e-5


def test_factor_f32_with_one_pass_bases_past_128_columns():
    """Figure 5 at l = 200 (q = 3) on a spectrum with a gap at k and a flat tail past it: every intermediate
    basis is well conditioned (the column-scaled Frobenius condition bound of the six panels is 204 to 289 in
    FP64, below the 1e3 of the one-pass test), so each takes a single CholeskyQR pass, with the bound formed
    from the blocked factor and the first apply writing the basis.  The factors match the FP64 oracle, which
    orthonormalises every basis fully, to the FP32 bar of the other cases."""
    m, n, k, p, q = 3000, 2000, 180, 20, 3
    sigma = np.concatenate([np.ones(k), np.full(300, 0.5)])
    A64 = gen.low_rank_matrix(m, n, sigma, 1e-3 / math.sqrt(n), seed=91)
    A32 = A64.astype(np.float32)
    G = gen.gaussian_matrix(n, k + p, seed=92)
    ref = orc.rsvd(A32.astype(np.float64), G, q)
    refk = ref.truncate(k)
    U, S, V, info = run_factor(A32, k, p, q, "f32", omega=G)
    assert info.status == 0
    assert max_rel_sigma(S, refk.D, k) <= 1e-4
    relgap = (ref.D[k - 1] - ref.D[k]) / ref.D[0]
    tol = 50 * math.sqrt(max(m, n)) * U32 / relgap
    assert subspace_sin(U, refk.U) <= tol
    assert subspace_sin(V, refk.V) <= tol
    assert orth_error(U) <= 1e-5 and orth_error(V) <= 1e-5


def test_exact_low_rank_input_drops_dependent_directions():
    """rank(A) = 5 < l = 16: the leading five triplets are exact (Section 4),
    the remaining singular values are zero or at rounding level."""
    sigma = np.array([5.0, 4.0, 3.0, 2.0, 1.0])
    A = gen.low_rank_matrix(400, 300, sigma, 0.0, seed=5)
    G = gen.gaussian_matrix(300, 16, seed=6)
    U, S, V, info = run_factor(A, 10, 6, 1, "f64", omega=G)
    assert np.allclose(S[:5], sigma, rtol=1e-12)
    assert np.all(S[5:] <= 1e-12)
    ref = orc.rsvd(A, G, 1)
    assert subspace_sin(U[:, :5], ref.U[:, :5]) < 1e-10
    assert np.linalg.norm(A - (U * S) @ V.T, 2) < 1e-12


def test_rank_l_flag_and_determinism():
    from paper_1607_01649_amd import RSVD_RETURN_RANK_L
    sigma = gen.spectrum("poly", 100, alpha=1.0)
    A = gen.low_rank_matrix(900, 700, sigma, 1e-6, seed=8).astype(np.float32)
    G = gen.gaussian_matrix(700, 30, seed=9)
    U1, S1, V1, info = run_factor(A, 20, 10, 1, "f32", omega=G, flags=RSVD_RETURN_RANK_L)
    assert info.rank_out == 30 and U1.shape == (900, 30) and V1.shape == (700, 30)
    U2, S2, V2, _ = run_factor(A, 20, 10, 1, "f32", omega=G, flags=RSVD_RETURN_RANK_L)
    assert np.array_equal(U1, U2) and np.array_equal(S1, S2) and np.array_equal(V1, V2)
    ref = orc.rsvd(A.astype(np.float64), G, 1)
    assert max_rel_sigma(S1, ref.D, 30) <= 1e-4
    # Stage B is exact (Remark in Section 3): at rank l, A^T U = V diag(S)
    assert np.max(np.abs(A.astype(np.float64).T @ U1 - V1 * S1)) <= 1e-4 * S1[0]


def test_nan_input_is_reported():
    A = np.ones((200, 100), dtype=np.float32)
    A[17, 3] = np.nan
    with pytest.raises(RuntimeError, match="NONFINITE"):
        run_factor(A, 5, 5, 0, "f32")


BF16_CASES = [
    # m, n, rank, alpha, k, p, q, sketch, proj
    (3000, 1500, 300, 0.5, 20, 10, 2, "bf16", "bf16"),
    (1237, 901, 200, 1.0, 12, 8, 1, "bf16", "f32"),
    (2048, 1024, 256, 0.5, 50, 14, 2, "bf16", "bf16"),
    # fewer row blocks than resident workgroups: both products split the contraction
    (20000, 2048, 256, 0.5, 96, 14, 1, "bf16", "bf16"),
]


@pytest.mark.parametrize("m,n,rank,alpha,k,p,q,sk,pj", BF16_CASES)
def test_factor_bf16_matches_the_quantisation_aware_oracle(m, n, rank, alpha, k, p, q, sk, pj):
    """bf16 operands, FP32 accumulation: parity against the oracle run on the
    identically rounded operands (differences are accumulation error only);
    the error of the format itself against the plain oracle is reported."""
    from oracle import quant
    sigma = gen.spectrum("poly", rank, alpha=alpha)
    A32 = gen.low_rank_matrix(m, n, sigma, 1e-3 / math.sqrt(n), seed=m + 5 * n).astype(np.float32)
    G = gen.gaussian_matrix(n, k + p, seed=m * n + 1)
    qa = quant.rsvd_quantized(A32, G, q, sk, pj)
    plain = orc.rsvd(A32.astype(np.float64), G, q)
    U, S, V, info = run_factor(A32, k, p, q, "f32", omega=G, sketch_dtype=sk, proj_dtype=pj)
    assert info.status == 0
    assert max_rel_sigma(S, qa.D, k) <= 1e-4
    relgap = (qa.D[k - 1] - qa.D[k]) / qa.D[0]
    assert subspace_sin(U, qa.U[:, :k]) <= 50 * math.sqrt(max(m, n)) * U32 / relgap
    print(f"bf16 format error vs plain oracle: max rel sigma {max_rel_sigma(S, plain.D, k):.2e}")
    assert max_rel_sigma(S, plain.D, k) <= 2e-2


FP8_CASES = [
    # m, n, rank, alpha, k, p, q, sketch, proj
    (3000, 1500, 300, 0.5, 20, 10, 2, "fp8", "fp8"),
    (1237, 901, 200, 1.0, 12, 8, 1, "fp8", "f32"),
    (2048, 1024, 256, 0.5, 50, 14, 2, "fp8", "fp8"),
    # FP8 sketch with a bf16 projection (two low-precision copies of A)
    (3000, 1500, 300, 0.5, 20, 10, 2, "fp8", "bf16"),
    # m mod 256 in [1, 128]: the last row block has waves wholly past the last row
    (1068, 700, 200, 1.0, 16, 8, 1, "fp8", "fp8"),
]


@pytest.mark.parametrize("m,n,rank,alpha,k,p,q,sk,pj", FP8_CASES)
def test_factor_fp8_matches_the_quantisation_aware_oracle(m, n, rank, alpha, k, p, q, sk, pj):
    """Block-scaled FP8 operands (128 x 128 tiles of A, 128-row segments of the
    thin operands), FP32 accumulation: parity against the oracle run on the
    identically quantised operands.  Beyond accumulation error, a thin-operand
    entry whose FP32 (GPU) and FP64 (oracle) values straddle a rounding
    boundary can land one E4M3 step apart, hence 1e-3 rather than the bf16
    case's 1e-4; the format error against the plain oracle is reported."""
    from oracle import quant
    sigma = gen.spectrum("poly", rank, alpha=alpha)
    A32 = gen.low_rank_matrix(m, n, sigma, 1e-3 / math.sqrt(n), seed=m + 5 * n).astype(np.float32)
    G = gen.gaussian_matrix(n, k + p, seed=m * n + 1)
    qa = quant.rsvd_quantized(A32, G, q, sk, pj)
    plain = orc.rsvd(A32.astype(np.float64), G, q)
    U, S, V, info = run_factor(A32, k, p, q, "f32", omega=G, sketch_dtype=sk, proj_dtype=pj)
    assert info.status == 0
    assert max_rel_sigma(S, qa.D, k) <= 1e-3
    print(f"fp8 format error vs plain oracle: max rel sigma {max_rel_sigma(S, plain.D, k):.2e}")
    assert max_rel_sigma(S, plain.D, k) <= 0.1


def test_factor_fp8_at_l520_matches_the_quantisation_aware_oracle():
    """The 65536^2 workload's shape of the method (k = 500, p = 20, q = 3,
    exponential decay sigma_j = exp(-j/150)) at 6000 x 5000: l = 520 takes
    three 192-column groups per FP8 product, the blocked Cholesky and the
    block Jacobi, all on FP8-derived data; m mod 256 = 112 puts waves past the
    last row.  Against the oracle on identically quantised operands the
    singular values agree to 1e-3 sigma_1 (a normwise gate: one-step E4M3
    differences in thin operands whose FP32 and FP64 values straddle a
    rounding boundary perturb B by a small multiple of 2^-4 of those entries);
    the format error against the plain FP64 oracle is reported."""
    from oracle import quant
    m, n, k, p, q = 6000, 5000, 500, 20, 3
    sigma = gen.spectrum("exp", 1000, tau=150.0)
    A32 = gen.low_rank_matrix(m, n, sigma, 1e-3 / math.sqrt(n), seed=61).astype(np.float32)
    G = gen.gaussian_matrix(n, k + p, seed=62)
    print(f"case fp8 l=520 {m}x{n}", flush=True)
    U, S, V, info = run_factor(A32, k, p, q, "f32", omega=G, sketch_dtype="fp8", proj_dtype="fp8")
    assert info.status == 0 and info.jacobi_sweeps >= 1
    qa = quant.rsvd_quantized(A32, G, q, "fp8", "fp8")
    plain = orc.rsvd(A32.astype(np.float64), G, q)
    norm_err = float(np.max(np.abs(S[:k] - qa.D[:k]))) / qa.D[0]
    print(f"fp8 l=520: max |sigma - sigma_qa| / sigma_1 = {norm_err:.2e}, "
          f"max rel vs qa {max_rel_sigma(S, qa.D, k):.2e}, format error vs plain {max_rel_sigma(S, plain.D, k):.2e}")
    assert norm_err <= 1e-3
    assert max_rel_sigma(S, plain.D, k) <= 0.1
    # the factors are orthonormal to FP32 accuracy and reproduce the rank-k residual of the oracle
    assert orth_error(U) <= 1e-4 and orth_error(V) <= 1e-4


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_rank_deficient_input(dtype):
    """A of exact rank 10 (small integers, so Y = A Omega with an integer
    Omega is exact) with k + p = 30: the Gram matrices of CholeskyQR are
    exactly singular.  Nothing fails; with FP32 data the dependent columns
    fall below the pivot threshold (l u^2 G_jj) and are dropped (counted), and
    the basis spans the range of A: the ten nonzero singular values are exact
    to rounding, the others vanish (columns of U and V past the rank are zero
    when dropped)."""
    g = np.random.default_rng(4)
    m, n, r, k, p = 500, 400, 10, 20, 10
    A = (g.integers(-2, 3, (m, r)) @ g.integers(-2, 3, (r, n))).astype(np.float64)
    omega = g.integers(-2, 3, (n, k + p)).astype(np.float64)
    s_true = np.linalg.svd(A, compute_uv=False)
    assert s_true[r - 1] > 1.0 and s_true[r] < 1e-10 * s_true[0]
    Ain = A if dtype == "f64" else A.astype(np.float32)
    U, S, V, info = run_factor(Ain, k, p, 1, dtype, omega=omega)
    assert info.status == 0
    tol = 1e-12 if dtype == "f64" else 1e-5
    assert max_rel_sigma(S, s_true, r) <= tol
    assert np.all(np.abs(S[r:k]) <= tol * S[0])
    Ut = np.linalg.svd(A)[0][:, :r]
    assert subspace_sin(Ut, U[:, :r]) <= (1e-10 if dtype == "f64" else 1e-4)
    assert np.linalg.norm(A - (U * S) @ V.T, 2) <= tol * S[0]
    if dtype == "f32":
        assert info.dropped_cols >= k + p - r
        assert np.all(U[:, r:k] == 0.0) and np.all(S[r:k] == 0.0)


def test_factor_at_l200_is_capturable_in_a_graph():
    """With eps = 0 and no info requested, rsvd_factor enqueues everything on
    the plan's stream without a host synchronisation, also at l > 128 (blocked
    Cholesky and block Jacobi): the call captures into a HIP graph, and every
    replay reproduces the eager result bit for bit."""
    import torch
    from paper_1607_01649_amd import RSVD, rsvd_factor
    dev = device()
    m, n, k, p, q = 1500, 1200, 190, 10, 1
    sigma = gen.spectrum("poly", 600, alpha=0.5)
    A = torch.from_numpy(gen.low_rank_matrix(m, n, sigma, 1e-6, seed=8).astype(np.float32)).to(dev)
    s = torch.cuda.Stream(dev)
    with torch.cuda.stream(s):
        solver = RSVD(m, n, k, p, q, dtype="f32", device=dev, seed=11)
        U = torch.zeros(m, k, dtype=torch.float32, device=dev)
        S = torch.zeros(k, dtype=torch.float64, device=dev)
        V = torch.zeros(n, k, dtype=torch.float32, device=dev)
        st, _ = rsvd_factor(solver.plan, A, U, S, V, want_info=False)
        assert st == 0
    s.synchronize()
    ref = (U.clone(), S.clone(), V.clone())
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=s):
        st2, _ = rsvd_factor(solver.plan, A, U, S, V, want_info=False)
    assert st2 == 0
    for rep in range(3):
        U.zero_(); S.zero_(); V.zero_()
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(U, ref[0]) and torch.equal(S, ref[1]) and torch.equal(V, ref[2]), rep
    ref_o = orc.rsvd_seeded(A.double().cpu().numpy(), k, p, q, seed=11)
    assert max_rel_sigma(S.cpu().numpy(), ref_o.D, k) <= 1e-4


# ---------------------------------------------------------------- certificate and fallback

def _cert_case(seed=95, m=700, n=500, tau=10.0):
    sigma = gen.spectrum("exp", 300, tau=tau)
    return gen.low_rank_matrix(m, n, sigma, 0.0, seed=seed)


@pytest.mark.parametrize("s", [0, 1])
def test_certificate_matches_the_oracle(s):
    """Section 14: bound = 10 sqrt(2/pi) max_i ||(A - U D V^T) g_i|| with the
    probes drawn from the same seed on both sides; with eps loose enough the
    rank-k result is accepted as is."""
    A = _cert_case()
    k, p, q, seed = 12, 8, 1, 5
    # eps far above the bound: accepted at rank k on both sides, bounds compared
    ref = orc.factor(A, k, p, q, seed, eps=100.0, n_probe=10, est_power=s)
    assert ref.certified and ref.rank == k
    U, S, V, info = run_factor(A, k, p, q, "f64", seed=seed, eps=100.0, n_probe=10, est_power=s)
    assert info.status == 0 and info.rank_out == k and info.fallback_steps == 0
    assert abs(info.err_bound - ref.bound) <= 1e-8 * ref.bound
    assert max_rel_sigma(S, ref.D, k) <= 1e-10
    true = np.linalg.norm(A - (U * S) @ V.T, 2)
    assert info.err_bound >= true


@pytest.mark.parametrize("dtype,sk,pj,b,eps", [("f64", "f64", "f64", 8, 1e-4), ("f32", "f32", "f32", 16, 1e-4),
                                               ("f32", "bf16", "f32", 8, 5e-2)])
def test_fallback_grows_to_the_tolerance_like_the_oracle(dtype, sk, pj, b, eps):
    """The rank-k result misses eps; the blocked range finder of Figure 12
    grows the basis (columns continuing Omega's sequence, two projections per
    block) until the Section 14 certificate holds, as the oracle does.  A bf16
    sketch only has to span; the projection B = Q^T A stays FP32 here, since
    its rounding error enters the residual the certificate measures.  With a
    bf16 sketch the basis follows bf16(A): the residual keeps the rounding
    A - bf16(A), which is full rank with a flat spectrum, so a probe sees its
    Frobenius norm (about 3.9e-3 sigma_1 here), and with the certificate's
    factor 10 sqrt(2/pi) the bound stalls near 3e-2 sigma_1 (about 0.03 at
    150 columns in an FP64 simulation of the bf16 sketch); that case runs at
    eps = 5e-2 and may need more columns than the exact basis."""
    A = _cert_case(seed=96)
    k, p, q, seed = 10, 5, 1, 7
    sk_, pj_ = sk, pj
    ref = orc.factor(A, k, p, q, seed, eps=eps, block=b, max_rank=150)
    assert ref.certified and ref.fallback_steps > 0
    Ain = A if dtype == "f64" else A.astype(np.float32)
    U, S, V, info = run_factor(Ain, k, p, q, dtype, seed=seed, eps=eps, fallback_block=b, max_rank=150,
                               sketch_dtype=sk_, proj_dtype=pj_)
    assert info.status == 0
    if dtype == "f64":
        assert info.rank_out == ref.rank and info.fallback_steps == ref.fallback_steps
        assert abs(info.err_bound - ref.bound) <= 1e-6 * ref.bound
        r = ref.rank
        assert max_rel_sigma(S, ref.D, min(r, 40)) <= 1e-9
    elif sk == "f32":
        assert abs(info.rank_out - ref.rank) <= b
    else:
        # the rounding floor makes the bf16 basis grow further than the exact one
        assert ref.rank - b <= info.rank_out <= 150
    true = np.linalg.norm(A - (U * S) @ V.T, 2)
    assert true <= eps * S[0] * 1.01
    assert info.err_bound <= eps * info.sigma1
    assert info.err_bound >= true * (1 - 1e-6)
    # Section 12.4: the downdated Frobenius residual matches the direct one
    QB_res = np.linalg.norm(A - (U * S) @ V.T)
    assert abs(info.frob_residual - QB_res) <= 1e-3 * np.linalg.norm(A) + 1e-6


def test_not_certified_when_the_rank_cap_is_reached():
    A = _cert_case(seed=97)
    U, S, V, info = run_factor(A, 10, 5, 0, "f64", seed=3, eps=1e-8, fallback_block=8, max_rank=31)
    assert info.status == 1                 # RSVD_NOT_CERTIFIED: factors written, tolerance missed
    assert info.rank_out == 31 and info.fallback_steps == 2
    assert info.err_bound > 1e-8 * info.sigma1
    ref = orc.factor(A, 10, 5, 0, 3, eps=1e-8, block=8, max_rank=31)
    assert ref.rank == 31 and not ref.certified
    assert max_rel_sigma(S, ref.D, 31) <= 1e-9


# ---------------------------------------------------------------- batched compression

def _batched_case(nblk, seed=1, lo=64, hi=512):
    import torch
    ms, ns = gen.batched_blocks(nblk, seed, lo, hi)
    host = [gen.kernel_block(int(ms[b]), int(ns[b]), seed, b) for b in range(nblk)]
    dev = [torch.from_numpy(K).to(device()) for K in host]
    return host, dev


def test_batched_compression_matches_the_per_block_oracle():
    """Every block is compressed to 1e-6 relative tolerance (Sections 12-14);
    ranks, basis widths and singular values follow the oracle run with the
    same per-block random streams; the true error meets the tolerance."""
    import torch
    from oracle.batched import compress_block
    from paper_1607_01649_amd import Batched
    nblk = 48
    host, dev = _batched_case(nblk)
    bt = Batched(dev, eps=1e-6, rank_cap=64, seed=42)
    bt.run()
    torch.cuda.synchronize()
    status = bt.status.cpu().numpy()
    ranks = bt.rank.cpu().numpy()
    assert np.all(status == 0)
    agree = 0
    for b in range(nblk):
        ref = compress_block(host[b], 1e-6, 42, b)
        U, S, V = (t.double().cpu().numpy() for t in bt.factors(b))
        agree += int(ranks[b] == ref.rank)
        r = min(ranks[b], ref.rank)
        assert np.max(np.abs(S[:r] - ref.S[:r]) / ref.S[0]) <= 1e-6
        K = host[b].astype(np.float64)
        s1 = np.linalg.svd(K, compute_uv=False)[0]
        assert np.linalg.norm(K - (U * S) @ V.T, 2) <= 1e-6 * s1
        assert np.linalg.norm(U.T @ U - np.eye(U.shape[1])) <= 1e-5
    assert agree >= nblk - 2


def test_batched_graph_replay_and_invalid_blocks():
    import torch
    from paper_1607_01649_amd import Batched
    host, dev = _batched_case(20, seed=3)
    dev[5] = torch.zeros(600, 100, device=device())        # more than 512 rows: rejected per block
    bt = Batched(dev, eps=1e-6, rank_cap=32, seed=9)
    bt.run()
    torch.cuda.synchronize()
    U0, S0, st0 = bt.U.clone(), bt.S.clone(), bt.status.clone()
    assert int(st0[5]) == -1 and int(bt.rank[5]) == 0
    assert all(int(st0[b]) == 0 for b in range(20) if b != 5)
    s = torch.cuda.Stream(device=device())
    bt.U.zero_()
    bt.S.zero_()
    torch.cuda.synchronize()
    bt.capture(s)
    for _ in range(3):
        bt.replay(s)
        s.synchronize()
        assert torch.equal(bt.S, S0) and torch.equal(bt.U, U0)
        bt.U.zero_()
        torch.cuda.synchronize()


def _batched_outputs(bt):
    return [t.clone() for t in (bt.U, bt.V, bt.S, bt.rank, bt.status)]


def test_batched_tile_variants_are_bit_identical():
    """Every MFMA tile shape consumes the k-slices in the same order, so all
    variants reproduce the default's outputs bit for bit (blocks from 16 to
    512 rows and columns: all four size classes, ragged tiles)."""
    import torch
    from paper_1607_01649_amd import Batched, RSVD_BATCHED_TILE_VARIANTS
    host, dev = _batched_case(24, seed=5, lo=16, hi=512)
    bt = Batched(dev, eps=1e-6, rank_cap=64, seed=11)
    for t in (bt.U, bt.V, bt.S):       # columns past rank_b are never written
        t.fill_(7.0)
    bt.run()
    torch.cuda.synchronize()
    ref = _batched_outputs(bt)
    assert all(int(s) in (0, 1) for s in ref[4].cpu())
    for v in range(RSVD_BATCHED_TILE_VARIANTS):
        for t in (bt.U, bt.V, bt.S):
            t.fill_(7.0)
        bt.tiles = [v, (v + 1) % RSVD_BATCHED_TILE_VARIANTS, (v + 3) % RSVD_BATCHED_TILE_VARIANTS, v]
        bt.run()
        torch.cuda.synchronize()
        got = _batched_outputs(bt)
        for a, b in zip(got, ref):
            assert torch.equal(a, b), f"tiles {bt.tiles}"


def test_batched_autotune_picks_valid_tiles_and_keeps_results():
    import torch
    from paper_1607_01649_amd import Batched, RSVDError, RSVD_BATCHED_TILE_VARIANTS
    host, dev = _batched_case(40, seed=6, lo=16, hi=400)      # classes 0..3 (400 > 384)
    bt = Batched(dev, eps=1e-6, rank_cap=64, seed=3)
    bt.run()
    torch.cuda.synchronize()
    ref = _batched_outputs(bt)
    tiles, ms = bt.autotune()
    assert len(tiles) == 4 and all(0 <= t < RSVD_BATCHED_TILE_VARIANTS for t in tiles)
    mx = [max(int(m), int(n)) for m, n in zip(bt.m.cpu(), bt.n.cpu())]
    for c in range(4):
        present = any((x - 1) // 128 == c for x in mx)
        assert all((t > 0) == present for t in ms[c]), (c, ms[c])
        if present:
            assert ms[c][tiles[c]] == min(ms[c])
    bt.run()
    torch.cuda.synchronize()
    for a, b in zip(_batched_outputs(bt), ref):
        assert torch.equal(a, b)
    s = torch.cuda.Stream(device=device())
    bt.U.zero_()
    torch.cuda.synchronize()
    bt.capture(s)
    bt.replay(s)
    s.synchronize()
    assert torch.equal(bt.U, ref[0]) and torch.equal(bt.S, ref[2])
    bt.tiles = [0, 0, 0, RSVD_BATCHED_TILE_VARIANTS]
    with pytest.raises(RSVDError):
        bt.run()
