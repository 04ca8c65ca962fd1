"""fpp_query_ex_noalloc (no allocation inside the library; static device scratch) against
fpp_query_ex through the C ABI: two calls in a row, the second with a smaller input, for the FP32
and BF16 + rerank paths, one call spanning several chunks of the scratch, and one index large
enough that its overflow dedup bitmaps are used."""
import numpy as np
import pytest

import synthdata

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def F():
    import paper_2206_01382_amd as F
    assert torch.cuda.is_available()
    F.lib()
    return F


def _same(a, b):
    assert torch.equal(a[0], b[0])
    assert torch.equal(a[1].view(torch.int32), b[1].view(torch.int32))


@pytest.mark.parametrize("store", ["fp32", "bf16"])
def test_noalloc_equals_query_ex_twice_second_smaller(F, store):
    X, Q = synthdata.clustered_sphere(20_000, 128, 300, 50, 0.3, seed=7)
    Xd, Qd = torch.from_numpy(X).cuda(), torch.from_numpy(Q).cuda()
    h = F.fpp_build_index(Xd, 6, 32, 0.3, 3, 1234, l=2, stores=("bf16",))
    try:
        for m, k, qp in ((300, 10, 48), (37, 100, 200)):
            Qm = Qd[:m].contiguous()
            ref = F.fpp_query(h, Qm, k, qp, store=store, stats=True)
            got = F.fpp_query_ex_noalloc(h, Qm, k, qp, store=store, stats=True)
            torch.cuda.synchronize()
            _same(got, ref)
            assert torch.equal(got[2], ref[2])
    finally:
        F.fpp_free_index(h)


def test_noalloc_many_chunks_and_bitmap_dedup(F):
    """The headline table shape (L = 100, l = 2, D = 128 at d = 128): 153.6 KB of list scratch
    per query, so 1,500 queries take several chunks of the static array; then qProbes = 20,000,
    where queries hold more distinct candidates than the LDS set and deduplicate in the bitmaps;
    then a smaller call again."""
    X, Q = synthdata.clustered_sphere(60_000, 128, 1_500, 100, 0.3, seed=8)
    Xd, Qd = torch.from_numpy(X).cuda(), torch.from_numpy(Q).cuda()
    h = F.fpp_build_index(Xd, 100, 128, 0.3, 3, 42, l=2)
    try:
        for m, qp in ((1_500, 50), (300, 20_000), (20, 50)):
            Qm = Qd[:m].contiguous()
            ref = F.fpp_query(h, Qm, 10, qp, stats=True)
            got = F.fpp_query_ex_noalloc(h, Qm, 10, qp, stats=True)
            torch.cuda.synchronize()
            _same(got, ref)
            assert torch.equal(got[2], ref[2])
            if qp == 20_000:
                assert int(ref[2][:, 2].max()) > 3072     # the bitmap path ran
    finally:
        F.fpp_free_index(h)


def test_noalloc_rejects_stage_timers(F):
    X, Q = synthdata.clustered_sphere(2_000, 16, 4, 5, 0.4, seed=9)
    Xd, Qd = torch.from_numpy(X).cuda(), torch.from_numpy(Q).cuda()
    h = F.fpp_build_index(Xd, 2, 8, 0.5, 1, 5, l=2)
    try:
        from paper_2206_01382_amd import _lib
        import ctypes
        ids = torch.empty((4, 3), dtype=torch.int32, device="cuda")
        sc = torch.empty((4, 3), dtype=torch.float32, device="cuda")
        st = np.zeros(4)
        o = _lib.fpp_query_opts(0, 0, None, st.ctypes.data_as(_lib.c_vp), 0)
        rc = _lib.lib().fpp_query_ex_noalloc(h, _lib.c_vp(Qd.data_ptr()), 4, 3, 8, ctypes.byref(o),
                                             _lib.c_vp(ids.data_ptr()), _lib.c_vp(sc.data_ptr()), None)
        assert rc == F.FPP_EINVAL
    finally:
        F.fpp_free_index(h)
