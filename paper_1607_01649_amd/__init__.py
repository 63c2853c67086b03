"""MI355X (gfx950) randomized range finder and randomized SVD.

Python binding of the C ABI in include/rsvd.h.  The functions named like the
C entry points marshal torch tensors (device memory) and the current HIP
stream into the library; all computation runs in the HIP kernels of
``librsvd.so``.  There is no CPU fallback: if the library is not built,
importing the binding raises.
"""
from __future__ import annotations

import ctypes
from typing import Optional

import torch

from . import _lib
from ._lib import (  # noqa: F401
    RSVD_BATCHED_CLASSES, RSVD_BATCHED_TILE_VARIANTS, RSVD_BF16, RSVD_E_ARG, RSVD_E_HIP, RSVD_E_NONFINITE, RSVD_E_UNSUPPORTED, RSVD_E_WORKSPACE,
    RSVD_F32, RSVD_F64, RSVD_FP8_E4M3, RSVD_MLP_NPARAM, RSVD_NOT_CERTIFIED, RSVD_OK, RSVD_RETURN_RANK_L,
    RSVD_ID_CUR, RSVD_NYSTROM, RSVD_SEL_NQ, RSVD_SEL_P, RSVD_SINGLE_PASS, RSVD_SINGLE_PASS_SYM, RSVD_SKETCH_SRHT,
    RSVD_TIMING, RSVDError, STREAM_CERT, STREAM_OMEGA, STREAM_PROBE, rsvd_desc, rsvd_info,
    status_str,
)

_DTYPES = {"f64": RSVD_F64, "f32": RSVD_F32, "bf16": RSVD_BF16, "fp8": RSVD_FP8_E4M3}
_TORCH = {RSVD_F64: torch.float64, RSVD_F32: torch.float32}


def _code(dt) -> int:
    if isinstance(dt, str):
        return _DTYPES[dt]
    if dt is torch.float64:
        return RSVD_F64
    if dt is torch.float32:
        return RSVD_F32
    return int(dt)


def _ptr(t: Optional[torch.Tensor]):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _stream_handle(device=None, stream=None):
    s = stream if stream is not None else torch.cuda.current_stream(device)
    return ctypes.c_void_p(s.cuda_stream)


def make_desc(m, n, k, p=10, q=1, a_dtype="f32", sketch_dtype=None, proj_dtype=None, seed=0, eps=0.0,
              n_probe=0, est_power=0, fallback_block=0, max_rank=0, flags=0) -> rsvd_desc:
    a = _code(a_dtype)
    d = rsvd_desc()
    d.m, d.n, d.k, d.p, d.q = int(m), int(n), int(k), int(p), int(q)
    d.a_dtype = a
    d.sketch_dtype = a if sketch_dtype is None else _code(sketch_dtype)
    d.proj_dtype = a if proj_dtype is None else _code(proj_dtype)
    d.seed = int(seed) & 0xFFFFFFFFFFFFFFFF
    d.eps = float(eps)
    d.n_probe, d.est_power = int(n_probe), int(est_power)
    d.fallback_block, d.max_rank = int(fallback_block), int(max_rank)
    d.flags = int(flags)
    return d


def rsvd_status_str(status: int) -> str:
    return status_str(status)


def rsvd_workspace_size(desc: rsvd_desc) -> int:
    out = ctypes.c_size_t(0)
    st = _lib.lib().rsvd_workspace_size(ctypes.byref(desc), ctypes.byref(out))
    if st != RSVD_OK:
        raise RSVDError(st, "rsvd_workspace_size")
    return int(out.value)


def rsvd_plan(desc: rsvd_desc, workspace: torch.Tensor, stream=None) -> ctypes.c_void_p:
    h = ctypes.c_void_p()
    st = _lib.lib().rsvd_plan(ctypes.byref(desc), _ptr(workspace), workspace.numel() * workspace.element_size(),
                              _stream_handle(workspace.device, stream), ctypes.byref(h))
    if st != RSVD_OK:
        raise RSVDError(st, "rsvd_plan")
    return h


def rsvd_factor(plan, A: torch.Tensor, U: torch.Tensor, S: torch.Tensor, V: Optional[torch.Tensor],
                omega: Optional[torch.Tensor] = None, want_info: bool = True):
    """Returns (status, rsvd_info or None).  A, U, V row-major (2-D, unit
    column stride); omega, if given, n x (k+p) float64 row-major."""
    info = rsvd_info() if want_info else None
    st = _lib.lib().rsvd_factor(plan, _ptr(A), A.stride(0), _ptr(omega), _ptr(U), U.stride(0), _ptr(S), _ptr(V),
                                V.stride(0) if V is not None else 0, ctypes.byref(info) if info is not None else None)
    return st, info


def rsvd_factor_noalloc(desc: rsvd_desc, A: torch.Tensor, U: torch.Tensor, S: torch.Tensor,
                        V: Optional[torch.Tensor], omega: Optional[torch.Tensor] = None, stream=None) -> int:
    """The fixed-rank factorisation in the library's own per-device workspace
    (no plan, no allocation); returns the status."""
    return _lib.lib().rsvd_factor_noalloc(ctypes.byref(desc), _ptr(A), A.stride(0), _ptr(omega), _ptr(U),
                                          U.stride(0), _ptr(S), _ptr(V), V.stride(0) if V is not None else 0,
                                          _stream_handle(A.device, stream))


def rsvd_k_srht_sketch(A: torch.Tensor, l: int, seed: int, stream=None):
    """The structured sketch of Section 6 on its own: returns (Y, signs, subset) with Y = A Omega (m x l),
    the signs (n) and the column subset (l, int32), computed by the library's kernels."""
    m, n = A.shape
    prec = RSVD_F64 if A.dtype == torch.float64 else RSVD_F32
    Y = torch.empty(m, l, dtype=A.dtype, device=A.device)
    sg = torch.empty(n, dtype=A.dtype, device=A.device)
    sub = torch.empty(l, dtype=torch.int32, device=A.device)
    st = _lib.lib().rsvd_k_srht_sketch(prec, m, n, _ptr(A), A.stride(0), int(l), int(seed) & 0xFFFFFFFFFFFFFFFF,
                                       _ptr(sg), _ptr(sub), _ptr(Y), Y.stride(0), _stream_handle(A.device, stream))
    if st != RSVD_OK:
        raise RSVDError(st, "rsvd_k_srht_sketch")
    return Y, sg, sub


def rsvd_destroy(plan) -> None:
    _lib.lib().rsvd_destroy(plan)


def rsvd_gaussian(seed: int, stream_id: int, out: torch.Tensor, col0: int = 0, stream=None) -> None:
    rows, cols = out.shape
    st = _lib.lib().rsvd_gaussian(int(seed), int(stream_id), rows, cols, int(col0), _code(out.dtype), _ptr(out),
                                  out.stride(0), _stream_handle(out.device, stream))
    if st != RSVD_OK:
        raise RSVDError(st, "rsvd_gaussian")


def rsvd_philox4x32_10(ctr: torch.Tensor, k0: int, k1: int, out: torch.Tensor, stream=None) -> None:
    """ctr, out: int32 device tensors of shape (count, 4) holding uint32 words."""
    st = _lib.lib().rsvd_philox4x32_10(ctr.shape[0], _ptr(ctr), int(k0) & 0xFFFFFFFF, int(k1) & 0xFFFFFFFF,
                                       _ptr(out), _stream_handle(out.device, stream))
    if st != RSVD_OK:
        raise RSVDError(st, "rsvd_philox4x32_10")


def rsvd_selector_set(plan, theta: torch.Tensor, tau: float) -> None:
    st = _lib.lib().rsvd_selector_set(plan, _ptr(theta), float(tau))
    if st != RSVD_OK:
        raise RSVDError(st, "rsvd_selector_set")


def rsvd_probe_sigma(plan, A: torch.Tensor, sigma16: torch.Tensor, x: Optional[torch.Tensor] = None) -> None:
    st = _lib.lib().rsvd_probe_sigma(plan, _ptr(A), A.stride(0), _ptr(sigma16), _ptr(x))
    if st != RSVD_OK:
        raise RSVDError(st, "rsvd_probe_sigma")


def rsvd_prefix_bounds(plan, A: torch.Tensor, widths) -> list:
    w = (ctypes.c_int32 * len(widths))(*[int(v) for v in widths])
    b = (ctypes.c_double * len(widths))()
    st = _lib.lib().rsvd_prefix_bounds(plan, _ptr(A), A.stride(0), len(widths), w, b)
    if st != RSVD_OK:
        raise RSVDError(st, "rsvd_prefix_bounds")
    return list(b)


def rsvd_mlp_forward(theta, X, H1, H2, Z, stream=None) -> None:
    st = _lib.lib().rsvd_mlp_forward(_ptr(theta), X.shape[0], _ptr(X), _ptr(H1), _ptr(H2), _ptr(Z),
                                     _stream_handle(X.device, stream))
    if st != RSVD_OK:
        raise RSVDError(st, "rsvd_mlp_forward")


def rsvd_mlp_backward(theta, X, H1, H2, Z, Y, M, grad, loss, scratch, stream=None) -> None:
    st = _lib.lib().rsvd_mlp_backward(_ptr(theta), X.shape[0], _ptr(X), _ptr(H1), _ptr(H2), _ptr(Z), _ptr(Y),
                                      _ptr(M), _ptr(grad), _ptr(loss), _ptr(scratch), _stream_handle(X.device, stream))
    if st != RSVD_OK:
        raise RSVDError(st, "rsvd_mlp_backward")


def rsvd_mlp_adam(theta, grad, m, v, lr, step, beta1=0.9, beta2=0.999, eps=1e-8, stream=None) -> None:
    st = _lib.lib().rsvd_mlp_adam(_ptr(theta), _ptr(grad), _ptr(m), _ptr(v), theta.numel(), float(lr), float(beta1),
                                  float(beta2), float(eps), int(step), _stream_handle(theta.device, stream))
    if st != RSVD_OK:
        raise RSVDError(st, "rsvd_mlp_adam")


def _aligned_workspace(nbytes: int, device) -> torch.Tensor:
    ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
    off = (-ws.data_ptr()) % 256
    return ws[off:off + nbytes]


def selector_grid_cap(m: int, n: int) -> int:
    return min(m, n, 1024)


class RSVD:
    """A plan plus its torch-allocated workspace for one problem shape.

    ``RSVD(m, n, k, p, q, dtype)(A)`` returns (U, S, V, info) with U (m x r),
    S (r, float64, descending), V (n x r) on A's device.  ``p = q = -1``
    makes a selector-mode plan: attach the network with ``set_selector``."""

    def __init__(self, m, n, k, p=10, q=1, dtype="f32", device="cuda", **kw):
        self.desc = make_desc(m, n, k, p, q, a_dtype=dtype, **kw)
        self.device = torch.device(device)
        nbytes = rsvd_workspace_size(self.desc)
        self.workspace = _aligned_workspace(nbytes, self.device)
        self.plan = rsvd_plan(self.desc, self.workspace)
        if p == -1 and q == -1:
            cap = selector_grid_cap(m, n)
            l = max(k + pp for pp in RSVD_SEL_P if k + pp <= cap)
        else:
            l = self.desc.k + self.desc.p
        self.rank_cap = max(l, self.desc.max_rank) if self.desc.eps > 0 else (
            l if (self.desc.flags & RSVD_RETURN_RANK_L) else self.desc.k)
        self.tdtype = _TORCH[self.desc.a_dtype]
        self.theta = None

    def set_selector(self, theta: torch.Tensor, tau: float = 0.5) -> None:
        self.theta = theta
        rsvd_selector_set(self.plan, theta, tau)

    def __call__(self, A: torch.Tensor, omega: Optional[torch.Tensor] = None, want_info: bool = True,
                 out=None, allow_not_certified: bool = True):
        r = self.rank_cap
        if out is None:
            U = torch.empty(self.desc.m, r, dtype=self.tdtype, device=self.device)
            S = torch.empty(r, dtype=torch.float64, device=self.device)
            V = torch.empty(self.desc.n, r, dtype=self.tdtype, device=self.device)
        else:
            U, S, V = out
        st, info = rsvd_factor(self.plan, A, U, S, V, omega, want_info or self.desc.eps > 0)
        if st < 0 or (st == RSVD_NOT_CERTIFIED and not allow_not_certified):
            raise RSVDError(st, "rsvd_factor")
        if info is not None:
            k = info.rank_out
            return U[:, :k], S[:k], V[:, :k], info
        return U, S, V, None

    def row_id(self, A: torch.Tensor, omega: Optional[torch.Tensor] = None, want_info: bool = True):
        """Randomized row ID (plan made with RSVD_ID_CUR): returns (I_s (k, int32), X (m x k), info) with
        A ~= X A(I_s, :)."""
        k = self.desc.k
        Is = torch.empty(k, dtype=torch.int32, device=self.device)
        X = torch.empty(self.desc.m, k, dtype=self.tdtype, device=self.device)
        info = rsvd_info() if want_info else None
        st = _lib.lib().rsvd_row_id(self.plan, _ptr(A), A.stride(0), _ptr(omega), _ptr(Is), _ptr(X), X.stride(0),
                                    ctypes.byref(info) if info is not None else None)
        if st < 0:
            raise RSVDError(st, "rsvd_row_id")
        return Is, X, info

    def cur(self, A: torch.Tensor, want_info: bool = True):
        """Randomized CUR (plan made with RSVD_ID_CUR): returns (J_s, U (k x k, float64), I_s, info) with
        A ~= A(:, J_s) U A(I_s, :)."""
        k = self.desc.k
        Js = torch.empty(k, dtype=torch.int32, device=self.device)
        Is = torch.empty(k, dtype=torch.int32, device=self.device)
        U = torch.empty(k, k, dtype=torch.float64, device=self.device)
        info = rsvd_info() if want_info else None
        st = _lib.lib().rsvd_cur(self.plan, _ptr(A), A.stride(0), _ptr(Js), _ptr(U), U.stride(0), _ptr(Is),
                                 ctypes.byref(info) if info is not None else None)
        if st < 0:
            raise RSVDError(st, "rsvd_cur")
        return Js, U, Is, info

    def __del__(self):
        p = getattr(self, "plan", None)
        if p is not None:
            try:
                rsvd_destroy(p)
            except Exception:
                pass
            self.plan = None


class Batched:
    """Batched compression of a list of FP32 blocks (device tensors, 2-D,
    unit column stride) to relative tolerance `eps`: device arrays of shapes,
    pointers, output offsets and the workspace are built once; `run()`
    launches rsvd_batched, `capture()` records it into a HIP graph and
    `replay()` launches the graph.  Outputs: U (sum m_b x rank_cap),
    V (sum n_b x rank_cap), S (nblk x rank_cap), rank, status.  `tiles`
    (one MFMA tile variant per size class, None = library default) is set
    by hand or by `autotune()` and applies to later run() / capture()."""

    def __init__(self, blocks, eps=1e-6, rank_cap=64, seed=0, n_workgroups=0, stream=None, tiles=None):
        self.blocks = list(blocks)
        dev = self.blocks[0].device
        self.device = dev
        nb = len(self.blocks)
        ms = [b.shape[0] for b in self.blocks]
        ns = [b.shape[1] for b in self.blocks]
        self.m = torch.tensor(ms, dtype=torch.int32, device=dev)
        self.n = torch.tensor(ns, dtype=torch.int32, device=dev)
        self.lda = torch.tensor([b.stride(0) for b in self.blocks], dtype=torch.int32, device=dev)
        self.ptrs = torch.tensor([b.data_ptr() for b in self.blocks], dtype=torch.int64, device=dev)
        offu = [0]
        offv = [0]
        for mm, nn in zip(ms, ns):
            offu.append(offu[-1] + mm * rank_cap)
            offv.append(offv[-1] + nn * rank_cap)
        self.offU = torch.tensor(offu[:-1], dtype=torch.int64, device=dev)
        self.offV = torch.tensor(offv[:-1], dtype=torch.int64, device=dev)
        self.U = torch.zeros(offu[-1], dtype=torch.float32, device=dev)
        self.V = torch.zeros(offv[-1], dtype=torch.float32, device=dev)
        self.S = torch.zeros(nb, rank_cap, dtype=torch.float64, device=dev)
        self.rank = torch.zeros(nb, dtype=torch.int32, device=dev)
        self.status = torch.zeros(nb, dtype=torch.int32, device=dev)
        self.eps, self.rank_cap, self.seed, self.nwg = float(eps), int(rank_cap), int(seed), int(n_workgroups)
        nbytes = ctypes.c_size_t(0)
        st = _lib.lib().rsvd_batched_workspace_size(nb, self.nwg, ctypes.byref(nbytes))
        if st != RSVD_OK:
            raise RSVDError(st, "rsvd_batched_workspace_size")
        ws = torch.empty(nbytes.value + 256, dtype=torch.uint8, device=dev)
        off = (-ws.data_ptr()) % 256
        self.ws = ws[off:off + nbytes.value]
        self.stream = stream
        self.graph = None
        self.tiles = None if tiles is None else [int(t) for t in tiles]

    def _head(self):
        return (len(self.blocks), _ptr(self.m), _ptr(self.n), _ptr(self.ptrs), _ptr(self.lda), self.eps,
                self.rank_cap, self.seed, _ptr(self.U), _ptr(self.S), _ptr(self.V), _ptr(self.offU),
                _ptr(self.offV), _ptr(self.rank), _ptr(self.status), self.nwg)

    def _tiles_arg(self):
        if self.tiles is None:
            return None
        if len(self.tiles) != _lib.RSVD_BATCHED_CLASSES:
            raise ValueError(f"tiles needs {_lib.RSVD_BATCHED_CLASSES} entries")
        return ctypes.cast((ctypes.c_int32 * len(self.tiles))(*self.tiles), ctypes.c_void_p)

    def _args(self):
        return self._head() + (self._tiles_arg(), _ptr(self.ws), self.ws.numel())

    def run(self):
        st = _lib.lib().rsvd_batched(*self._args(), _stream_handle(self.device, self.stream))
        if st != RSVD_OK:
            raise RSVDError(st, "rsvd_batched")

    def autotune(self):
        """Time every tile variant per size class (rsvd_batched_autotune), keep
        the fastest in `tiles`; returns (tiles, ms) with ms[class][variant]."""
        nc, nv = _lib.RSVD_BATCHED_CLASSES, _lib.RSVD_BATCHED_TILE_VARIANTS
        out = (ctypes.c_int32 * nc)()
        ms = (ctypes.c_float * (nc * nv))()
        st = _lib.lib().rsvd_batched_autotune(*self._head(), _ptr(self.ws), self.ws.numel(),
                                              _stream_handle(self.device, self.stream),
                                              ctypes.cast(out, ctypes.c_void_p), ctypes.cast(ms, ctypes.c_void_p))
        if st != RSVD_OK:
            raise RSVDError(st, "rsvd_batched_autotune")
        self.tiles = list(out)
        return self.tiles, [list(ms[c * nv:(c + 1) * nv]) for c in range(nc)]

    def capture(self, stream):
        h = ctypes.c_void_p()
        st = _lib.lib().rsvd_batched_graph_create(*self._args(), ctypes.c_void_p(stream.cuda_stream),
                                                  ctypes.byref(h))
        if st != RSVD_OK:
            raise RSVDError(st, "rsvd_batched_graph_create")
        self.graph = h

    def replay(self, stream):
        st = _lib.lib().rsvd_graph_launch(self.graph, ctypes.c_void_p(stream.cuda_stream))
        if st != RSVD_OK:
            raise RSVDError(st, "rsvd_graph_launch")

    def factors(self, b):
        """(U_b, S_b, V_b) of block b (host copies, rank columns)."""
        r = int(self.rank[b])
        mm, nn = self.blocks[b].shape
        ou, ov = int(self.offU[b]), int(self.offV[b])
        U = self.U[ou:ou + mm * self.rank_cap].view(mm, self.rank_cap)[:, :r]
        V = self.V[ov:ov + nn * self.rank_cap].view(nn, self.rank_cap)[:, :r]
        return U, self.S[b, :r], V

    def __del__(self):
        if getattr(self, "graph", None) is not None:
            try:
                _lib.lib().rsvd_graph_destroy(self.graph)
            except Exception:
                pass
            self.graph = None
