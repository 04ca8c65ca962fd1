"""Serving loop (continuous batching) through the C ABI: every request's result equals the same
query run alone and the oracle's answer, admission by scratch bytes neither loses nor duplicates
requests, requests larger than the pool are rejected, a failing batch fails only its own requests,
and timestamps are consistent."""
import time

import numpy as np
import pytest

import synthdata
from _parity import check_topk, swap_budget
from oracle import falconn as O

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


X_SERVE, Q_SERVE = None, None


@pytest.fixture(scope="module")
def env():
    import paper_2206_01382_amd as F
    global X_SERVE, Q_SERVE
    assert torch.cuda.is_available()
    X_SERVE, Q_SERVE = synthdata.clustered_sphere(30_000, 64, 300, 40, 0.3, seed=11)
    Xd, Qd = torch.from_numpy(X_SERVE).cuda(), torch.from_numpy(Q_SERVE).cuda()
    h = F.fpp_build_index(Xd, 8, 32, 0.3, 3, 77, l=2, stores=("bf16",))
    yield F, h, Xd, Qd
    F.fpp_free_index(h)


@pytest.fixture(scope="module")
def oracle_index(env):
    return O.build_index(X_SERVE, 8, 32, 0.3, 3, 77, l=2)


def _requests(rng, m_total, n_req, ks, qps):
    reqs = []
    row = 0
    for _ in range(n_req):
        m = int(rng.integers(1, 17))
        if row + m > m_total:
            row = 0
        reqs.append((row, m, int(rng.choice(ks)), int(rng.choice(qps))))
        row += m
    return reqs


def _run(F, sv, Qd, reqs, kmax, pace_s=0.0):
    # the server's streams are not ordered after torch's: the sentinel fills must be done before
    # the first submission, or a late fill could overwrite a served result
    outs = [(torch.full((m, k), -7, dtype=torch.int32, device="cuda"),
             torch.full((m, k), 7.0, dtype=torch.float32, device="cuda")) for (_, m, k, _) in reqs]
    torch.cuda.synchronize()
    tickets = []
    for (row, m, k, qp), (ids, sc) in zip(reqs, outs):
        q = Qd[row:row + m]
        tickets.append(F.fpp_server_submit(sv, q.data_ptr(), m, k, qp, ids.data_ptr(), sc.data_ptr()))
        if pace_s:
            time.sleep(pace_s)
    stamps = [F.fpp_server_wait(sv, t, 60_000) for t in tickets]
    return outs, stamps, tickets


@pytest.mark.parametrize("store", ["fp32", "bf16"])
def test_results_alone_equal_results_in_the_mix(env, oracle_index, store):
    """Served in mixed batches, each request equals the same query run alone (bit-identical)
    and the oracle's answer (FP32: Algorithm 1 and FP64 scores; BF16: the FP64 rerank of the
    short list of max(100, 2k) by the approximate score), under the comparison rule."""
    F, h, Xd, Qd = env
    rng = np.random.default_rng(1)
    reqs = _requests(rng, Qd.shape[0], 120, (1, 10, 100), (8, 40, 200))
    sv = F.fpp_server_create(h, scratch_bytes=256 << 20, n_streams=3, max_batch=64, store=store)
    try:
        outs, stamps, _ = _run(F, sv, Qd, reqs, 100)
        st = F.fpp_server_get_stats(sv)
    finally:
        F.fpp_server_destroy(sv)
    assert st["completed"] == len(reqs) and st["failed"] == 0
    assert st["batches"] < len(reqs)              # requests were batched together
    swaps = results = 0
    for (row, m, k, qp), (ids, sc), (status, ts, td) in zip(reqs, outs, stamps):
        assert status == 0 and 0 < ts <= td
        ri, rs = F.fpp_query(h, Qd[row:row + m].contiguous(), k, qp, store=store)
        assert torch.equal(ids, ri) and torch.equal(sc, rs)
        Qr = Q_SERVE[row:row + m]
        if store == "fp32":
            oi, osc, _ = O.query(oracle_index, Qr, k, qp)
        else:
            oi, osc, _ = O.query_reranked(oracle_index, Qr, k, qp, R=max(100, 2 * k), storage=store)
        swaps += check_topk(X_SERVE, Qr, ids.cpu().numpy(), sc.cpu().numpy(), oi, osc)
        results += m * k
    assert swaps <= swap_budget(results), swaps


def test_small_pool_admission_and_oversized_requests(env):
    F, h, Xd, Qd = env
    pool = 64 << 10      # a few small batches fit; a 16-query request with all probes does not
    sv = F.fpp_server_create(h, scratch_bytes=pool, n_streams=4, max_batch=16)
    try:
        rng = np.random.default_rng(2)
        reqs = [(int(r), int(m), 10, 40) for r, m in zip(rng.integers(0, Qd.shape[0] - 4, size=60),
                                                         rng.integers(1, 5, size=60))]
        outs, stamps, tickets = _run(F, sv, Qd, reqs, 10)
        st = F.fpp_server_get_stats(sv)
        assert st["completed"] == 60 and st["failed"] == 0
        assert 0 < st["scratch_high_water"] <= pool
        assert len(set(tickets)) == 60
        for (row, m, k, qp), (ids, sc) in zip(reqs, outs):
            ri, rs = F.fpp_query(h, Qd[row:row + m].contiguous(), k, qp)
            assert torch.equal(ids, ri) and torch.equal(sc, rs)
        ids = torch.empty((17, 10), dtype=torch.int32, device="cuda")
        sc = torch.empty((17, 10), dtype=torch.float32, device="cuda")
        with pytest.raises(F.FppError) as e:    # needs more scratch than the pool holds
            F.fpp_server_submit(sv, Qd.data_ptr(), 16, 10, 10 ** 6, ids.data_ptr(), sc.data_ptr())
        assert e.value.code == F.FPP_ECAPACITY
        with pytest.raises(F.FppError) as e:    # more queries than one launch packs
            F.fpp_server_submit(sv, Qd.data_ptr(), 17, 10, 40, ids.data_ptr(), sc.data_ptr())
        assert e.value.code == F.FPP_ECAPACITY
        t = F.fpp_server_submit(sv, Qd.data_ptr(), 4, 10, 40, ids.data_ptr(), sc.data_ptr())
        assert F.fpp_server_wait(sv, t, 60_000)[0] == 0   # the loop keeps serving
    finally:
        F.fpp_server_destroy(sv)


def test_poll_reports_a_completed_ticket_once(env):
    F, h, Xd, Qd = env
    sv = F.fpp_server_create(h, scratch_bytes=64 << 20, n_streams=2, max_batch=16)
    try:
        ids = torch.empty((2, 10), dtype=torch.int32, device="cuda")
        sc = torch.empty((2, 10), dtype=torch.float32, device="cuda")
        t = F.fpp_server_submit(sv, Qd.data_ptr(), 2, 10, 40, ids.data_ptr(), sc.data_ptr())
        for _ in range(2000):
            st, ts, td = F.fpp_server_poll(sv, t)
            if st != 1:
                break
            time.sleep(0.001)
        assert st == 0 and td >= ts > 0
        with pytest.raises(F.FppError):
            F.fpp_server_poll(sv, t)
    finally:
        F.fpp_server_destroy(sv)


def test_overlapping_batches_on_several_streams(env):
    F, h, Xd, Qd = env
    sv = F.fpp_server_create(h, scratch_bytes=1 << 30, n_streams=4, max_batch=32)
    try:
        rng = np.random.default_rng(3)
        reqs = _requests(rng, Qd.shape[0], 400, (10,), (40, 400))
        outs, stamps, _ = _run(F, sv, Qd, reqs, 10)
        st = F.fpp_server_get_stats(sv)
    finally:
        F.fpp_server_destroy(sv)
    assert st["completed"] == 400 and st["max_inflight_batches"] >= 2
    for (row, m, k, qp), (ids, sc) in zip(reqs[::20], outs[::20]):
        ri, rs = F.fpp_query(h, Qd[row:row + m].contiguous(), k, qp)
        assert torch.equal(ids, ri) and torch.equal(sc, rs)


@pytest.mark.parametrize("store,probe_score", [("fp32", "gap"), ("simhash", "sum"), ("bf16", "gap")])
def test_served_options_equal_direct_queries(env, store, probe_score):
    """The server passes the store and the probe score through: each request equals the direct
    query with the same options."""
    F, h, Xd, Qd = env
    hh = h
    if store == "simhash":
        hh = F.fpp_build_index(Xd, 8, 32, 0.3, 3, 77, l=2, stores=("simhash",))
    try:
        rng = np.random.default_rng(4)
        reqs = _requests(rng, Qd.shape[0], 60, (1, 10), (8, 40, 200))
        sv = F.fpp_server_create(hh, scratch_bytes=256 << 20, n_streams=2, max_batch=64, store=store,
                                 probe_score=probe_score)
        try:
            outs, stamps, _ = _run(F, sv, Qd, reqs, 10)
        finally:
            F.fpp_server_destroy(sv)
        for (row, m, k, qp), (ids, sc), (status, ts, td) in zip(reqs, outs, stamps):
            assert status == 0
            ri, rs = F.fpp_query(hh, Qd[row:row + m].contiguous(), k, qp, store=store, probe_score=probe_score)
            assert torch.equal(ids, ri) and torch.equal(sc, rs)
    finally:
        if hh is not h:
            F.fpp_free_index(hh)


def test_replay_submits_on_schedule_and_matches_direct_queries(env):
    """The native load generator submits each request at its scheduled time; every result equals
    the same query run alone, and no request is submitted before its time."""
    F, h, Xd, Qd = env
    rng = np.random.default_rng(5)
    n = 80
    m = rng.integers(1, 17, size=n).astype(np.int32)
    k = rng.choice([1, 10], size=n).astype(np.int32)
    qp = rng.choice([8, 40, 200], size=n).astype(np.int32)
    q_row = np.array([int(rng.integers(0, Qd.shape[0] - 16)) for _ in range(n)], dtype=np.int64)
    out_off = np.concatenate([[0], np.cumsum(m.astype(np.int64) * k)[:-1]]).astype(np.int64)
    total = int((m.astype(np.int64) * k).sum())
    ids = torch.full((total,), -7, dtype=torch.int32, device="cuda")
    sc = torch.full((total,), 7.0, dtype=torch.float32, device="cuda")
    torch.cuda.synchronize()   # the server's streams are not ordered after torch's
    arrive = np.cumsum(rng.exponential(100_000, size=n)).astype(np.int64)   # ~0.1 ms apart
    sv = F.fpp_server_create(h, scratch_bytes=256 << 20, n_streams=2, max_batch=64)
    try:
        t0 = time.monotonic_ns() + 1_000_000
        tickets = F.fpp_server_replay(sv, Qd.data_ptr(), t0, arrive, q_row, m, k, qp, ids.data_ptr(),
                                      sc.data_ptr(), out_off)
        stamps = [F.fpp_server_wait(sv, int(t), 60_000) for t in tickets.tolist()]
        # a request the server rejects (more queries than one launch packs) stops the replay there
        with pytest.raises(F.FppError) as e:
            F.fpp_server_replay(sv, Qd.data_ptr(), time.monotonic_ns(), [0, 0], [0, 0], [65, 1], [1, 1],
                                [8, 8], ids.data_ptr(), sc.data_ptr(), [0, 0])
        assert e.value.code == F.FPP_ECAPACITY
    finally:
        F.fpp_server_destroy(sv)
    assert len(set(tickets.tolist())) == n and tickets.min() > 0
    for i, (status, ts, td) in enumerate(stamps):
        assert status == 0 and ts >= t0 + arrive[i] and td >= ts
        r, mm, kk, o = int(q_row[i]), int(m[i]), int(k[i]), int(out_off[i])
        ri, rs = F.fpp_query(h, Qd[r:r + mm].contiguous(), kk, int(qp[i]))
        assert torch.equal(ids[o:o + mm * kk].view(mm, kk), ri)
        assert torch.equal(sc[o:o + mm * kk].view(mm, kk), rs)


def test_failed_batch_fails_only_its_requests(env):
    """A batch that fails on the device side (forced from the host after its first kernel is on
    the stream) completes its requests with FPP_EHIP and returns its scratch; the loop then
    serves later requests correctly."""
    F, h, Xd, Qd = env
    sv = F.fpp_server_create(h, scratch_bytes=64 << 20, n_streams=2, max_batch=16)
    try:
        ids = torch.full((3, 10), -7, dtype=torch.int32, device="cuda")
        sc = torch.full((3, 10), 7.0, dtype=torch.float32, device="cuda")
        torch.cuda.synchronize()
        F.fpp_server_debug_fail_batches(sv, 1)
        t = F.fpp_server_submit(sv, Qd.data_ptr(), 3, 10, 40, ids.data_ptr(), sc.data_ptr())
        st, ts, td = F.fpp_server_wait(sv, t, 60_000)
        assert st == F.FPP_EHIP and td >= ts > 0
        stats = F.fpp_server_get_stats(sv)
        assert stats["failed"] == 1 and stats["completed"] == 0
        reqs = [(r, 2, 10, 40) for r in range(0, 40, 2)]
        outs, stamps, _ = _run(F, sv, Qd, reqs, 10)
        stats = F.fpp_server_get_stats(sv)
        assert stats["completed"] == len(reqs) and stats["failed"] == 1
        for (row, m, k, qp), (i2, s2), (status, _, _) in zip(reqs, outs, stamps):
            assert status == 0
            ri, rs = F.fpp_query(h, Qd[row:row + m].contiguous(), k, qp)
            assert torch.equal(i2, ri) and torch.equal(s2, rs)
        with pytest.raises(F.FppError):
            F.fpp_server_debug_fail_batches(sv, -1)
    finally:
        F.fpp_server_destroy(sv)
