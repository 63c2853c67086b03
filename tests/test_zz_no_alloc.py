"""rsvd_factor_noalloc (the entry point for callers that cannot allocate)
against rsvd_plan + rsvd_factor on the same description and input: the same
kernels in a different workspace, so the factors must agree bit for bit.
Two calls in a row, the second on a smaller input, so that contents left in
the library's array by the first call cannot leak into the second."""
import numpy as np
import pytest

from tests.gpu_helpers import device
from workloads import gen

pytestmark = pytest.mark.gpu

CASES = [
    # (m, n, k, p, q, a_dtype, low-precision operands, seed)
    (2000, 2000, 20, 10, 1, "f64", None, 11),
    (700, 500, 12, 8, 1, "f64", None, 12),
    (3000, 2500, 100, 28, 2, "f32", None, 13),
    (1300, 900, 40, 10, 1, "f32", "bf16", 14),
]


def _inputs(m, n, dt, seed):
    import torch
    sigma = gen.spectrum("poly", min(m, n) // 2, alpha=1.0)
    A = gen.low_rank_matrix(m, n, sigma, 1e-6, seed=seed)
    return torch.from_numpy(A).to(device(), torch.float64 if dt == "f64" else torch.float32)


def _with_plan(A, m, n, k, p, q, dt, lp, seed):
    import torch
    from paper_1607_01649_amd import RSVD
    U, S, V, _ = RSVD(m, n, k, p, q, dtype=dt, device=device(), seed=seed, sketch_dtype=lp, proj_dtype=lp)(A)
    torch.cuda.synchronize()
    return U.clone(), S.clone(), V.clone()


def _no_alloc(A, m, n, k, p, q, dt, lp, seed):
    import torch
    from paper_1607_01649_amd import RSVD_OK, make_desc, rsvd_factor_noalloc
    d = make_desc(m, n, k, p, q, a_dtype=dt, sketch_dtype=lp, proj_dtype=lp, seed=seed)
    U = torch.full((m, k), float("nan"), dtype=A.dtype, device=A.device)
    S = torch.full((k,), float("nan"), dtype=torch.float64, device=A.device)
    V = torch.full((n, k), float("nan"), dtype=A.dtype, device=A.device)
    st = rsvd_factor_noalloc(d, A, U, S, V)
    torch.cuda.synchronize()
    assert st == RSVD_OK, st
    return U, S, V


@pytest.mark.parametrize("pair", [(0, 1), (2, 3)])
def test_no_alloc_matches_the_planned_call_twice_in_a_row(pair):
    import torch
    for idx in pair:                      # the second case of each pair is the smaller input
        m, n, k, p, q, dt, lp, seed = CASES[idx]
        print(f"no-alloc case m={m} n={n} k={k} p={p} q={q} {dt} {lp}", flush=True)
        A = _inputs(m, n, dt, seed)
        ref = _with_plan(A, m, n, k, p, q, dt, lp, seed)
        got = _no_alloc(A, m, n, k, p, q, dt, lp, seed)
        for name, r, g in zip("USV", ref, got):
            assert torch.isfinite(g).all(), name
            assert torch.equal(r, g), f"{name}: max diff {float((r.double() - g.double()).abs().max()):.3e}"
        S = got[1].cpu().numpy()
        assert np.all(np.diff(S) <= 0)


def test_no_alloc_refuses_what_does_not_fit_or_is_not_fixed_rank():
    import ctypes
    import torch
    from paper_1607_01649_amd import RSVD_E_ARG, RSVD_E_WORKSPACE, _lib, make_desc
    lib = _lib.lib()
    dev = device()
    buf = torch.zeros(1024, dtype=torch.float32, device=dev)
    ptr = ctypes.c_void_p(buf.data_ptr())
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    big = make_desc(20000, 20000, 100, 10, 2, a_dtype="f32")
    assert lib.rsvd_factor_noalloc(ctypes.byref(big), ptr, 20000, None, ptr, 100, ptr, None, 0, stream) == \
        RSVD_E_WORKSPACE
    cert = make_desc(700, 500, 12, 8, 1, a_dtype="f64", eps=1e-3, max_rank=40)
    assert lib.rsvd_factor_noalloc(ctypes.byref(cert), ptr, 500, None, ptr, 40, ptr, None, 0, stream) == RSVD_E_ARG
    sel = make_desc(700, 500, 12, -1, -1, a_dtype="f32")
    assert lib.rsvd_factor_noalloc(ctypes.byref(sel), ptr, 500, None, ptr, 12, ptr, None, 0, stream) == RSVD_E_ARG
    torch.cuda.synchronize()
