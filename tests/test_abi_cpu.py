"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every function include/rsvd.h declares, and rejects invalid arguments before
touching the device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", h) for h in ("rsvd.h", "rsvd_kernels.h")]


def _declared_functions():
    text = "".join(open(h).read() for h in HEADERS)
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(rsvd_[a-z0-9_]+)\s*\(", text)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    from paper_1607_01649_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.fail("librsvd.so is not built; run __graft_entry__.build()")
    return _lib.load()


def test_header_declares_the_boundary():
    names = _declared_functions()
    for want in ("rsvd_workspace_size", "rsvd_plan", "rsvd_factor", "rsvd_destroy", "rsvd_status_str",
                 "rsvd_gaussian", "rsvd_philox4x32_10"):
        assert want in names


def test_every_declared_symbol_is_exported(lib):
    from paper_1607_01649_amd import _lib
    bound = {name for name, _, _ in _lib.SIGNATURES}
    for name in _declared_functions():
        assert hasattr(lib, name), name
        assert name in bound, f"{name} has no Python binding"


def test_struct_layouts_match_the_header(lib):
    from paper_1607_01649_amd._lib import rsvd_desc, rsvd_info
    assert ctypes.sizeof(rsvd_desc) == 80
    assert ctypes.sizeof(rsvd_info) == 104
    assert rsvd_desc.seed.offset == 40 and rsvd_desc.eps.offset == 48 and rsvd_desc.flags.offset == 72
    assert rsvd_info.err_bound.offset == 24 and rsvd_info.stage_ms.offset == 40 and rsvd_info.nn_launches.offset == 80


def _desc(**kw):
    from paper_1607_01649_amd import make_desc
    base = dict(m=1000, n=800, k=20, p=10, q=1, a_dtype="f32")
    base.update(kw)
    return make_desc(**base)


def _ws(lib, d):
    n = ctypes.c_size_t(0)
    st = lib.rsvd_workspace_size(ctypes.byref(d), ctypes.byref(n))
    return st, n.value


def test_workspace_size_for_valid_descriptions(lib):
    for kw in (dict(), dict(a_dtype="f64"), dict(m=50000, n=20000, k=100, p=10, q=2),
               dict(m=517, n=389, k=7, p=6, q=0)):
        st, n = _ws(lib, _desc(**kw))
        assert st == 0 and n > 0
    # larger problems need more workspace
    assert _ws(lib, _desc(m=4000))[1] > _ws(lib, _desc(m=1000))[1]


@pytest.mark.parametrize("kw", [
    dict(k=0), dict(p=-1), dict(q=-1), dict(m=0), dict(n=-5),
    dict(k=790, p=20),                 # k + p > min(m, n)
    dict(eps=-1.0), dict(eps=float("nan")),
    dict(a_dtype=7), dict(max_rank=5),  # max_rank below k + p
    dict(n_probe=-1), dict(est_power=-2), dict(n_probe=65), dict(fallback_block=300),
])
def test_invalid_descriptions_are_rejected_on_the_host(lib, kw):
    st, _ = _ws(lib, _desc(**kw))
    assert st == -1
    h = ctypes.c_void_p()
    d = _desc(**kw)
    assert lib.rsvd_plan(ctypes.byref(d), ctypes.c_void_p(1 << 20), 1 << 30, None, ctypes.byref(h)) == -1
    assert not h.value


def test_unsupported_combinations(lib):
    st, _ = _ws(lib, _desc(a_dtype="f64", sketch_dtype="f32"))
    assert st == -5


def test_plan_checks_workspace_before_touching_the_device(lib):
    d = _desc()
    st, need = _ws(lib, d)
    h = ctypes.c_void_p()
    assert lib.rsvd_plan(ctypes.byref(d), None, need, None, ctypes.byref(h)) == -2
    assert lib.rsvd_plan(ctypes.byref(d), ctypes.c_void_p(4096), need - 1, None, ctypes.byref(h)) == -2
    assert lib.rsvd_plan(ctypes.byref(d), ctypes.c_void_p(4096 + 8), need, None, ctypes.byref(h)) == -2


def test_null_arguments(lib):
    assert lib.rsvd_workspace_size(None, None) == -1
    assert lib.rsvd_factor(None, None, 0, None, None, 0, None, None, 0, None) == -1
    assert lib.rsvd_gaussian(0, 4, 10, 10, 0, 1, None, 10, None) == -1
    assert lib.rsvd_gaussian(0, 4, 10, 10, 0, 9, ctypes.c_void_p(4096), 10, None) == -1
    assert lib.rsvd_philox4x32_10(-1, None, 0, 0, None, None) == -1
    lib.rsvd_destroy(None)
    assert lib.rsvd_status_str(-3) == b"RSVD_E_HIP"


def test_selector_mode_workspace_covers_every_grid_point(lib):
    from paper_1607_01649_amd._lib import RSVD_SEL_P
    st, need = _ws(lib, _desc(p=-1, q=-1, eps=1e-3, max_rank=800))
    assert st == 0
    for p in RSVD_SEL_P:
        if 20 + p <= 800:
            st2, n2 = _ws(lib, _desc(p=p, q=4, eps=1e-3, max_rank=800))
            assert st2 == 0 and n2 <= need
    assert _ws(lib, _desc(p=-1, q=0))[0] == -1 and _ws(lib, _desc(p=0, q=-1))[0] == -1


def test_selector_and_network_entries_reject_bad_arguments(lib):
    f = ctypes.c_void_p(4096)
    assert lib.rsvd_selector_set(None, f, 0.5) == -1
    assert lib.rsvd_probe_sigma(None, f, 10, f, None) == -1
    w = (ctypes.c_int32 * 1)(5)
    b = (ctypes.c_double * 1)()
    assert lib.rsvd_prefix_bounds(None, f, 10, 1, w, b) == -1
    assert lib.rsvd_mlp_forward(None, 4, f, f, f, f, None) == -1
    assert lib.rsvd_mlp_forward(f, 0, f, f, f, f, None) == -1
    assert lib.rsvd_mlp_backward(f, 4, f, f, f, f, f, f, f, f, None, None) == -1
    assert lib.rsvd_mlp_adam(f, f, f, f, 10, 1e-3, 0.9, 0.999, 1e-8, 0, None) == -1     # step must be >= 1
    assert lib.rsvd_mlp_adam(f, f, f, f, 10, 1e-3, 1.0, 0.999, 1e-8, 1, None) == -1     # beta1 < 1


def test_no_alloc_entry_checks_its_limits_before_touching_the_device(lib):
    f = ctypes.c_void_p(4096)
    big = _desc(m=20000, n=20000, k=100, p=10, q=2)
    assert lib.rsvd_factor_noalloc(ctypes.byref(big), f, 20000, None, f, 100, f, None, 0, None) == -2
    for kw in (dict(eps=1e-3, max_rank=40), dict(p=-1, q=-1), dict(flags=2), dict(k=0)):
        d = _desc(**kw)
        assert lib.rsvd_factor_noalloc(ctypes.byref(d), f, 800, None, f, 40, f, None, 0, None) == -1
    assert lib.rsvd_factor_noalloc(None, f, 800, None, f, 40, f, None, 0, None) == -1


def test_structured_sketch_rejected_where_not_supported(lib):
    from paper_1607_01649_amd import RSVD_SKETCH_SRHT
    for kw in (dict(m=100, n=40000), dict(m=100, n=20000, a_dtype="f64"), dict(m=100, n=500, sketch_dtype="bf16"),
               dict(m=100, n=500, p=-1, q=-1)):
        st, _ = _ws(lib, _desc(flags=RSVD_SKETCH_SRHT, **kw))
        assert st == -1, kw
    st, need = _ws(lib, _desc(m=100, n=500, flags=RSVD_SKETCH_SRHT))
    assert st == 0 and need > _ws(lib, _desc(m=100, n=500))[1]


def test_nystrom_needs_a_square_matrix_and_no_certificate(lib):
    from paper_1607_01649_amd import RSVD_NYSTROM
    assert _ws(lib, _desc(m=800, n=800, flags=RSVD_NYSTROM))[0] == 0
    for kw in (dict(m=1000, n=800), dict(m=800, n=800, eps=1e-3, max_rank=40), dict(m=800, n=800, p=-1, q=-1)):
        assert _ws(lib, _desc(flags=RSVD_NYSTROM, **kw))[0] == -1, kw


def test_single_pass_descriptions(lib):
    from paper_1607_01649_amd import (RSVD_NYSTROM, RSVD_RETURN_RANK_L, RSVD_SINGLE_PASS, RSVD_SINGLE_PASS_SYM,
                                      RSVD_SKETCH_SRHT)
    assert _ws(lib, _desc(q=0, flags=RSVD_SINGLE_PASS))[0] == 0
    assert _ws(lib, _desc(m=800, q=0, flags=RSVD_SINGLE_PASS_SYM))[0] == 0
    assert _ws(lib, _desc(q=0, sketch_dtype="bf16", proj_dtype="bf16", flags=RSVD_SINGLE_PASS))[0] == 0
    bad = [dict(q=1, flags=RSVD_SINGLE_PASS),
           dict(q=0, eps=1e-2, max_rank=40, flags=RSVD_SINGLE_PASS),
           dict(q=0, flags=RSVD_SINGLE_PASS | RSVD_SINGLE_PASS_SYM),
           dict(q=0, flags=RSVD_SINGLE_PASS_SYM),                      # m != n
           dict(q=0, flags=RSVD_SINGLE_PASS | RSVD_RETURN_RANK_L),
           dict(q=0, flags=RSVD_SINGLE_PASS | RSVD_SKETCH_SRHT),
           dict(m=800, q=0, flags=RSVD_SINGLE_PASS_SYM | RSVD_NYSTROM),
           dict(q=0, sketch_dtype="bf16", proj_dtype="f32", flags=RSVD_SINGLE_PASS),
           dict(q=0, sketch_dtype="fp8", proj_dtype="fp8", flags=RSVD_SINGLE_PASS),
           dict(p=-1, q=-1, flags=RSVD_SINGLE_PASS)]
    for kw in bad:
        assert _ws(lib, _desc(**kw))[0] == -1, kw


def test_id_cur_descriptions(lib):
    from paper_1607_01649_amd import RSVD_ID_CUR, RSVD_SINGLE_PASS
    assert _ws(lib, _desc(q=1, flags=RSVD_ID_CUR))[0] == 0
    assert _ws(lib, _desc(q=1, flags=RSVD_ID_CUR))[1] > _ws(lib, _desc(q=1))[1]
    bad = [dict(k=100, p=40, flags=RSVD_ID_CUR),                      # k + p > 128
           dict(eps=1e-2, max_rank=40, flags=RSVD_ID_CUR),
           dict(sketch_dtype="bf16", proj_dtype="bf16", flags=RSVD_ID_CUR),
           dict(q=0, flags=RSVD_ID_CUR | RSVD_SINGLE_PASS),
           dict(p=-1, q=-1, flags=RSVD_ID_CUR)]
    for kw in bad:
        assert _ws(lib, _desc(**kw))[0] == -1, kw
