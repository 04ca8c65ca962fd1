"""The C-ABI library: it loads, exports every entry point include/fpp.h declares, and its host-side
validation rejects bad arguments before touching a GPU (no compute call is made here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fpp.h")
LIB = os.path.join(ROOT, "paper_2206_01382_amd", "libfpp.so")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(fpp_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def so():
    if not os.path.exists(LIB):
        pytest.fail("libfpp.so is not built (run __graft_entry__.build())")
    return ctypes.CDLL(LIB)


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("fpp_build_index", "fpp_query", "fpp_free_index", "fpp_last_error",
                 "fpp_server_create", "fpp_server_submit", "fpp_query_batch"):
        assert must in names


def test_library_exports_every_declared_symbol(so):
    missing = [n for n in declared_functions() if not hasattr(so, n)]
    assert not missing, missing


def test_binding_covers_every_declared_symbol():
    from paper_2206_01382_amd import _lib
    assert sorted(_lib.SIGNATURES) == declared_functions()
    _lib.lib()   # binds every signature


def test_version_and_defaults(so):
    from paper_2206_01382_amd import _lib
    L = _lib.lib()
    assert b"gfx950" in L.fpp_version()
    o = _lib.fpp_build_opts()
    L.fpp_default_build_opts(ctypes.byref(o))
    assert (o.l, o.stores, o.keep_rounding, o.tables_per_pass) == (2, 0, 0, 0)
    q = _lib.fpp_query_opts()
    L.fpp_default_query_opts(ctypes.byref(q))
    assert (q.store, q.rerank_R) == (0, 0)
    s = _lib.fpp_server_opts()
    L.fpp_default_server_opts(ctypes.byref(s))
    assert s.n_streams >= 1 and s.max_batch >= 1 and s.scratch_bytes > 0


@pytest.mark.parametrize("args,code,msg", [
    # (n, d, L, D, alpha, iProbes)
    ((0, 64, 10, 64, 0.5, 1), -1, "n="),
    ((100, 0, 10, 64, 0.5, 1), -1, "d="),
    ((100, 2000, 10, 64, 0.5, 1), -1, "d="),
    ((100, 64, 0, 64, 0.5, 1), -1, "L="),
    ((100, 64, 10, 48, 0.5, 1), -1, "D=48"),
    ((100, 64, 10, 1, 0.5, 1), -1, "D=1"),
    ((100, 64, 10, 64, 0.0, 1), -1, "alpha"),
    ((100, 64, 10, 64, 1.5, 1), -1, "alpha"),
    ((100, 64, 10, 64, float("nan"), 1), -1, "alpha"),
    ((100, 64, 10, 64, 0.5, 0), -1, "iProbes"),
    ((100, 64, 10, 64, 0.5, 17), -1, "iProbes"),
    ((100, 4000, 10, 64, 0.5, 1), -1, "d="),
])
def test_build_argument_validation(args, code, msg):
    from paper_2206_01382_amd import _lib
    L = _lib.lib()
    n, d, Lt, D, a, ip = args
    h = ctypes.c_void_p()
    fake = ctypes.c_void_p(0x1000)   # never dereferenced: validation fails first
    rc = L.fpp_build_index(fake, n, d, Lt, D, a, ip, 1, ctypes.byref(h))
    assert rc == code
    assert msg in L.fpp_last_error().decode()
    assert not h.value


def test_build_null_x_and_l1_iprobes_limit():
    from paper_2206_01382_amd import _lib
    L = _lib.lib()
    h = ctypes.c_void_p()
    assert L.fpp_build_index(None, 10, 8, 1, 8, 0.5, 1, 1, ctypes.byref(h)) == -1
    o = _lib.fpp_build_opts(1, 0, 0, 0)      # l = 1: at most D buckets per point
    rc = L.fpp_build_index_ex(ctypes.c_void_p(0x1000), 10, 8, 1, 4, 0.5, 5, 1, ctypes.byref(o), None,
                              ctypes.byref(h))
    assert rc == -1 and "iProbes" in L.fpp_last_error().decode()
    o = _lib.fpp_build_opts(3, 0, 0, 0)
    rc = L.fpp_build_index_ex(ctypes.c_void_p(0x1000), 10, 8, 1, 4, 0.5, 1, 1, ctypes.byref(o), None,
                              ctypes.byref(h))
    assert rc == -1 and "l=3" in L.fpp_last_error().decode()


def test_query_null_index_rejected():
    from paper_2206_01382_amd import _lib
    L = _lib.lib()
    assert L.fpp_query(None, None, 1, 10, 10, None, None, None) == -1
    assert L.fpp_query_workspace_bytes(None, 1, 1, 1, None) == -1
    L.fpp_free_index(None)          # ignored
    L.fpp_server_destroy(None)      # ignored


def test_normal_quantile_matches_scipy(so):
    """The library's AS 241 quantile (used by the threshold filter) against scipy's ndtri."""
    from scipy.special import ndtri
    so.fpp_normal_quantile.restype = ctypes.c_double
    so.fpp_normal_quantile.argtypes = [ctypes.c_double]
    for p in (1e-300, 1e-50, 1e-12, 1e-6, 2.2e-3, 0.02425, 0.075, 0.3, 0.5, 0.7, 0.975, 1 - 1e-9):
        got, want = so.fpp_normal_quantile(p), float(ndtri(p))
        assert abs(got - want) <= 1e-14 * max(1.0, abs(want)), (p, got, want)
    assert so.fpp_normal_quantile(0.5) == 0.0
    assert so.fpp_normal_quantile(0.0) != so.fpp_normal_quantile(0.0)   # NaN outside (0, 1)


def test_build_option_validation():
    import paper_2206_01382_amd._lib as L
    lib = L.lib()
    o = L.fpp_build_opts()
    lib.fpp_default_build_opts(ctypes.byref(o))
    assert (o.kappa, o.center, o.filter, o.threshold) == (0, 0, L.FPP_FILTER_FRACTION, 0.0)
    h = ctypes.c_void_p()
    for field, val in (("kappa", -1), ("center", 2), ("filter", 7), ("threshold", float("inf"))):
        bad = L.fpp_build_opts()
        lib.fpp_default_build_opts(ctypes.byref(bad))
        setattr(bad, field, val)
        rc = lib.fpp_build_index_ex(ctypes.c_void_p(16), 100, 8, 2, 8, 0.5, 1, 1, ctypes.byref(bad),
                                    None, ctypes.byref(h))
        assert rc == L.FPP_EINVAL, field
