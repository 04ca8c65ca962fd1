"""GPU path (C ABI) against the CPU oracle, element by element, on seeded synthetic inputs.

Bar: hash lists, build records, CSR tables, probe sets and candidate counts are bit-exact;
float32 scores are within 1e-6 relative of the oracle's float64 dot products (1e-6 of
sum |q_j x_j| where |s| < 0.1); top-k ids are identical except at positions where the two ids'
float64 scores lie within twice that bound (adjudicated near-ties: counted, printed at the end of
the session, at most 0.1% of the compared positions).
"""
import json
import math
import os

import numpy as np
import pytest

import synthdata
from _parity import check_topk, score_tol, swap_budget
from golden.make_fullsize_oracle import probe_digest, table_digest
from oracle import falconn as O

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_2206_01382_amd as F
    F.lib()
    yield


def F():
    import paper_2206_01382_amd as F
    return F


# ----------------------------------------------------------------------------------------------
# configurations: (name, data kind, n, d, L, D, l, alpha, iProbes, m)
CONFIGS = {
    "c1_gauss_10k_d64": dict(kind="c1"),
    "l2_clustered": dict(kind="cl", n=20_000, d=128, L=6, D=32, l=2, alpha=0.3, iProbes=3, m=40,
                         centers=50, spread=0.3),
    "pad_d100_D16": dict(kind="cl", n=4_000, d=100, L=5, D=16, l=2, alpha=0.5, iProbes=2, m=30,
                         centers=20, spread=0.4),
    "wideD_d20_D64": dict(kind="cl", n=3_000, d=20, L=3, D=64, l=2, alpha=0.25, iProbes=4, m=30,
                          centers=10, spread=0.5),
    "p256_lanes2": dict(kind="cl", n=3_000, d=200, L=2, D=128, l=2, alpha=0.3, iProbes=3, m=20,
                        centers=10, spread=0.4),
    "p512_d300_D256": dict(kind="cl", n=2_000, d=300, L=2, D=256, l=2, alpha=0.2, iProbes=3, m=20,
                           centers=10, spread=0.4),
    "k16_iprobes10": dict(kind="cl", n=2_000, d=64, L=3, D=32, l=2, alpha=0.4, iProbes=10, m=20,
                          centers=10, spread=0.4),
    "l1_D8_iprobes3": dict(kind="cl", n=1_500, d=12, L=4, D=8, l=1, alpha=0.6, iProbes=3, m=20,
                           centers=5, spread=0.5),
    # many tables: probe totals up to L take the direct selection
    "manyL_d24_L40": dict(kind="cl", n=3_000, d=24, L=40, D=16, l=2, alpha=0.4, iProbes=2, m=20,
                          centers=10, spread=0.4),
    "l1_L24_D16": dict(kind="cl", n=2_000, d=16, L=24, D=16, l=1, alpha=0.5, iProbes=2, m=20,
                       centers=8, spread=0.5),
    # d not a multiple of 4: element loads in the hash kernels, ragged row chunks in the gather
    "odd_d30_D32": dict(kind="cl", n=2_500, d=30, L=3, D=32, l=2, alpha=0.4, iProbes=2, m=20,
                        centers=8, spread=0.4),
    # the fused hash-and-select kernel with items of 8 lanes (P = 128): D = P and D = P / 2
    "fused_d128_D128": dict(kind="cl", n=3_000, d=128, L=8, D=128, l=2, alpha=0.3, iProbes=3, m=30,
                            centers=10, spread=0.4),
    "fused_half_d100_D64": dict(kind="cl", n=3_000, d=100, L=8, D=64, l=2, alpha=0.3, iProbes=3, m=30,
                                centers=10, spread=0.4),
    # the largest sizes the boundary takes: d = 1024 (P = 1024, a whole wave per rotation) with 16
    # buckets per point, and D = 2048 (P = 2048) for l = 1
    "max_d1024_D1024_ip16": dict(kind="cl", n=3_000, d=1024, L=2, D=1024, l=2, alpha=0.5, iProbes=16,
                                 m=10, centers=4, spread=0.4),
    "max_D2048_l1_ip16": dict(kind="cl", n=1_500, d=48, L=2, D=2048, l=1, alpha=0.3, iProbes=16, m=10,
                              centers=6, spread=0.4),
}
SEED = 1234


def make(name):
    c = CONFIGS[name]
    if c["kind"] == "c1":
        w = synthdata.workload("c1_gauss_10k_d64")
        return dict(X=w.X, Q=w.Q, L=w.L, D=w.D, l=w.l, alpha=w.alpha, iProbes=w.iProbes)
    X, Q = synthdata.clustered_sphere(c["n"], c["d"], c["m"], c["centers"], c["spread"], seed=7)
    return dict(X=X, Q=Q, L=c["L"], D=c["D"], l=c["l"], alpha=c["alpha"], iProbes=c["iProbes"])


_cache = {}


def built(name):
    """(workload dict, oracle index, GPU handle, X on device, Q on device) — built once."""
    if name not in _cache:
        w = make(name)
        oi = O.build_index(w["X"], w["L"], w["D"], w["alpha"], w["iProbes"], SEED, l=w["l"])
        Xd = torch.from_numpy(w["X"]).cuda()
        Qd = torch.from_numpy(w["Q"]).cuda()
        h = F().fpp_build_index(Xd, w["L"], w["D"], w["alpha"], w["iProbes"], SEED, l=w["l"],
                                stores=("bf16", "fp8"))
        torch.cuda.synchronize()
        _cache[name] = (w, oi, h, Xd, Qd)
    return _cache[name]


# ----------------------------------------------------------------------------------------------
@pytest.mark.parametrize("name", list(CONFIGS))
def test_signs_match(name):
    w, oi, h, Xd, Qd = built(name)
    np.testing.assert_array_equal(F().fpp_debug_signs(h), oi.signs)


@pytest.mark.parametrize("name", list(CONFIGS))
def test_query_hash_lists_bit_exact(name):
    w, oi, h, Xd, Qd = built(name)
    V = np.concatenate([w["Q"], w["X"][:50]])
    a, c = F().fpp_debug_query_lists(h, torch.from_numpy(V).cuda())
    a, c = a.cpu().numpy(), c.cpu().numpy()
    for t in range(w["L"]):
        for f in range(w["l"]):
            hl = O.hash_lists(V, oi.signs[t, f], w["D"])
            np.testing.assert_array_equal(a[:, t, f].view(np.uint32), hl.a.view(np.uint32))
            np.testing.assert_array_equal(c[:, t, f], hl.code)


def _near_tie_vectors(d, rng):
    """Vectors whose projections tie exactly or nearly (equal in the leading bits): basis
    vectors, constant vectors, a*e0 + b*e1 with tiny b, repeated coordinates, zero."""
    out = [np.zeros(d), np.ones(d) / math.sqrt(d)]
    for i in (0, 1, d - 1):
        e = np.zeros(d)
        e[i] = 1.0
        out.append(e)
    for b in (1e-9, 1e-7, 3e-7, 1e-6, 4e-6, 1e-5, 1e-4, 1e-3):
        x = np.zeros(d)
        x[0], x[1] = 1.0, b
        out.append(x)
        y = np.zeros(d)
        y[0], y[1], y[min(2, d - 1)] = 1.0, b, -2.5 * b
        out.append(y)
    for _ in range(6):
        x = rng.standard_normal(d)
        x[rng.integers(0, d, size=d // 2)] = x[0]          # many equal coordinates
        out.append(x)
        z = rng.standard_normal(d)
        z = z + 1e-6 * rng.standard_normal(d)              # generic
        out.append(z)
    return np.stack(out).astype(np.float32)


@pytest.mark.parametrize("name", ["l2_clustered", "p512_d300_D256", "c1_gauss_10k_d64", "pad_d100_D16"])
def test_query_hash_lists_near_ties_bit_exact(name):
    """Lists whose |y| values tie exactly or agree in their leading bits (the order then rests
    on the full float bits and the index) are bit-exact."""
    w, oi, h, Xd, Qd = built(name)
    V = _near_tie_vectors(w["X"].shape[1], np.random.default_rng(5))
    a, c = F().fpp_debug_query_lists(h, torch.from_numpy(V).cuda())
    a, c = a.cpu().numpy(), c.cpu().numpy()
    for t in range(w["L"]):
        for f in range(w["l"]):
            hl = O.hash_lists(V, oi.signs[t, f], w["D"])
            np.testing.assert_array_equal(a[:, t, f].view(np.uint32), hl.a.view(np.uint32))
            np.testing.assert_array_equal(c[:, t, f], hl.code)


def test_query_hash_lists_d128_D128_bit_exact():
    """The headline shape (d = P = D = 128, l = 2) on random and near-tie vectors."""
    X, Q = synthdata.clustered_sphere(2_000, 128, 200, 20, 0.3, seed=21)
    Xd = torch.from_numpy(X).cuda()
    h = F().fpp_build_index(Xd, 4, 128, 0.3, 3, 99, l=2)
    try:
        V = np.concatenate([Q, _near_tie_vectors(128, np.random.default_rng(6))])
        a, c = F().fpp_debug_query_lists(h, torch.from_numpy(V).cuda())
        a, c = a.cpu().numpy(), c.cpu().numpy()
        S = O.rotation_signs(99, 4, 2, 128)
        for t in range(4):
            for f in range(2):
                hl = O.hash_lists(V, S[t, f], 128)
                np.testing.assert_array_equal(a[:, t, f].view(np.uint32), hl.a.view(np.uint32))
                np.testing.assert_array_equal(c[:, t, f], hl.code)
    finally:
        F().fpp_free_index(h)


@pytest.mark.parametrize("name", ["l2_clustered", "p512_d300_D256", "c1_gauss_10k_d64", "pad_d100_D16",
                                  "odd_d30_D32"])
def test_query_hash_list_prefix_bit_exact(name):
    """With W <= D / 2 stored entries the kernel finishes only the first D / 2 sorted keys (all
    D when an equal-key run crosses position D / 2): positions [0, W) are bit-exact on random and
    near-tie vectors, for W around that cut."""
    w, oi, h, Xd, Qd = built(name)
    D = w["D"]
    V = np.concatenate([w["Q"][:40], _near_tie_vectors(w["X"].shape[1], np.random.default_rng(7))])
    ref = {(t, f): O.hash_lists(V, oi.signs[t, f], D) for t in range(w["L"]) for f in range(w["l"])}
    for W in sorted({1, max(1, D // 4), max(1, D // 2 - 1), D // 2, D // 2 + 1, D}):
        a, c = F().fpp_debug_query_lists(h, torch.from_numpy(V).cuda(), W=W)
        a, c = a.cpu().numpy(), c.cpu().numpy()
        for (t, f), hl in ref.items():
            np.testing.assert_array_equal(a[:, t, f, :W].view(np.uint32), hl.a[:, :W].view(np.uint32))
            np.testing.assert_array_equal(c[:, t, f, :W], hl.code[:, :W])


def test_query_hash_list_prefix_d128_D128_bit_exact():
    """The headline shape with the headline prefix (qProbes = 50 reads 52 entries) and the
    prefixes around D / 2 = 64, on random vectors and on vectors with runs of equal keys."""
    X, Q = synthdata.clustered_sphere(2_000, 128, 200, 20, 0.3, seed=22)
    Xd = torch.from_numpy(X).cuda()
    h = F().fpp_build_index(Xd, 4, 128, 0.3, 3, 98, l=2)
    try:
        V = np.concatenate([Q, _near_tie_vectors(128, np.random.default_rng(8))])
        S = O.rotation_signs(98, 4, 2, 128)
        ref = {(t, f): O.hash_lists(V, S[t, f], 128) for t in range(4) for f in range(2)}
        for W in (1, 52, 63, 64, 65):
            a, c = F().fpp_debug_query_lists(h, torch.from_numpy(V).cuda(), W=W)
            a, c = a.cpu().numpy(), c.cpu().numpy()
            for (t, f), hl in ref.items():
                np.testing.assert_array_equal(a[:, t, f, :W].view(np.uint32), hl.a[:, :W].view(np.uint32))
                np.testing.assert_array_equal(c[:, t, f, :W], hl.code[:, :W])
        with pytest.raises(F().FppError):
            F().fpp_debug_query_lists(h, torch.from_numpy(V).cuda(), W=129)
    finally:
        F().fpp_free_index(h)


@pytest.mark.parametrize("P,l", [(2, 1), (2, 2), (4, 2), (8, 1), (8, 2)])
def test_query_hash_lists_tiny_P_bit_exact(P, l):
    """Rotations of 2 to 8 elements (one lane per item): whole lists and every prefix length."""
    rng = np.random.default_rng(P * 10 + l)
    X = rng.standard_normal((300, P)).astype(np.float32)
    X /= np.linalg.norm(X, axis=1, keepdims=True)
    h = F().fpp_build_index(torch.from_numpy(X).cuda(), 3, P, 0.5, 1, 97, l=l)
    try:
        V = np.concatenate([X[:30], _near_tie_vectors(P, np.random.default_rng(9))])
        S = O.rotation_signs(97, 3, l, P)
        ref = {(t, f): O.hash_lists(V, S[t, f], P) for t in range(3) for f in range(l)}
        for W in [None] + list(range(1, P + 1)):
            a, c = F().fpp_debug_query_lists(h, torch.from_numpy(V).cuda(), W=W)
            a, c = a.cpu().numpy(), c.cpu().numpy()
            n = P if W is None else W
            for (t, f), hl in ref.items():
                np.testing.assert_array_equal(a[:, t, f, :n].view(np.uint32), hl.a[:, :n].view(np.uint32))
                np.testing.assert_array_equal(c[:, t, f, :n], hl.code[:, :n])
    finally:
        F().fpp_free_index(h)


@pytest.mark.parametrize("name", list(CONFIGS))
def test_build_records_bit_exact(name):
    w, oi, h, Xd, Qd = built(name)
    for t in sorted({0, w["L"] - 1}):
        b, k = F().fpp_debug_build_records(h, t)
        torch.cuda.synchronize()
        lists = [O.hash_lists(w["X"], oi.signs[t, f], w["D"]) for f in range(w["l"])]
        ob, ok = O.top_pairs(lists, w["D"], w["iProbes"])
        np.testing.assert_array_equal(b.cpu().numpy().astype(np.int64), ob)
        np.testing.assert_array_equal(k.cpu().numpy().view(np.uint32), ok.view(np.uint32))


@pytest.mark.parametrize("d,D,l,ip", [(128, 128, 2, 3), (128, 128, 1, 1), (64, 32, 2, 10),
                                      (300, 256, 2, 3), (300, 256, 2, 16), (20, 16, 1, 4)])
def test_build_records_exact_ties_bit_exact(d, D, l, ip):
    """Build records of vectors whose projections tie exactly (basis, constant and repeated-
    coordinate vectors; zero), so equal |y| meet at the top-iProbes boundary and the list order
    rests on the index. For d = 128 the data also holds two points of the headline data set whose
    second function in table 6 of the seed-42 index ties at list positions 2 and 3 (the build
    once took the larger index first there)."""
    X = [_near_tie_vectors(d, np.random.default_rng(d + ip))]
    if d == 128:
        X.insert(0, synthdata.workload("c2_cluster_1m_d128").X[[648304, 786308]])
    X = np.concatenate(X).astype(np.float32)
    L = 8 if d != 128 else 100
    h = F().fpp_build_index(torch.from_numpy(X).cuda(), L, D, 0.5, ip, 42, l=l)
    try:
        S = O.rotation_signs(42, L, l, O.padded_dim(d, D))
        for t in range(L):
            b, k = F().fpp_debug_build_records(h, t)
            torch.cuda.synchronize()
            lists = [O.hash_lists(X, S[t, f], D) for f in range(l)]
            ob, ok = O.top_pairs(lists, D, ip)
            np.testing.assert_array_equal(b.cpu().numpy().astype(np.int64), ob, err_msg=f"table {t}")
            np.testing.assert_array_equal(k.cpu().numpy().view(np.uint32), ok.view(np.uint32))
    finally:
        F().fpp_free_index(h)


@pytest.mark.parametrize("name", list(CONFIGS))
def test_tables_bit_exact(name):
    w, oi, h, Xd, Qd = built(name)
    sizes = F().fpp_index_table_sizes(h)
    for t in range(w["L"]):
        off, ids = F().fpp_debug_export_table(h, t)
        np.testing.assert_array_equal(off, oi.offsets[t])
        np.testing.assert_array_equal(ids, oi.ids[t])
        assert sizes[t] == len(oi.ids[t])
    info = F().fpp_index_get_info(h)
    assert info["total_ids"] == sum(len(i) for i in oi.ids)
    assert info["max_bucket"] == max(int(np.max(np.diff(o))) for o in oi.offsets)


@pytest.mark.parametrize("name", list(CONFIGS))
def test_probe_sets_bit_exact(name):
    w, oi, h, Xd, Qd = built(name)
    total = w["L"] * (w["D"] ** w["l"])
    # totals up to L / 4 take the direct ranking of the sparse selection, larger ones the bisection
    for qp in sorted({1, 2, 17, max(1, w["L"] // 4), max(1, w["L"] // 2), w["L"], 4 * w["L"], 50 * w["L"],
                      total, total + 5}):
        g = F().fpp_debug_probes(h, Qd, qp).cpu().numpy()
        for r in range(w["Q"].shape[0]):
            ref = O.probes(oi, w["Q"][r], qp)
            assert sorted(g[r].tolist()) == sorted(ref.tolist()), (qp, r)


@pytest.mark.parametrize("name", ["l2_clustered", "c1_gauss_10k_d64", "manyL_d24_L40", "l1_L24_D16",
                                  "wideD_d20_D64", "fused_d128_D128", "fused_half_d100_D64"])
def test_probe_sets_near_ties_bit_exact(name):
    """Probe budgets up to 2L take the fused hash-and-select kernel; vectors whose projections
    tie (zero, constant, basis vectors) emit more outputs than it holds, so those queries are
    finished by the list-based kernels. Every probe set is bit-exact either way."""
    w, oi, h, Xd, Qd = built(name)
    V = np.concatenate([w["Q"][:10], _near_tie_vectors(w["X"].shape[1], np.random.default_rng(11))])
    Vd = torch.from_numpy(V).cuda()
    for qp in sorted({1, max(1, w["L"] // 2), w["L"], 2 * w["L"], 2 * w["L"] + 1}):
        g = F().fpp_debug_probes(h, Vd, qp).cpu().numpy()
        for r in range(V.shape[0]):
            ref = O.probes(oi, V[r], qp)
            assert sorted(g[r].tolist()) == sorted(ref.tolist()), (qp, r)


@pytest.mark.parametrize("name", ["c1_gauss_10k_d64", "l2_clustered", "p512_d300_D256", "l1_D8_iprobes3"])
def test_gap_probe_sets_bit_exact(name):
    """Plain Falconn's gap score: probe sets bit-exact, and queries match the oracle."""
    w, oi, h, Xd, Qd = built(name)
    total = w["L"] * (w["D"] ** w["l"])
    for qp in sorted({1, 3, max(1, w["L"] // 4), w["L"], 4 * w["L"], 50 * w["L"], total}):
        g = F().fpp_debug_probes(h, Qd, qp, probe_score="gap").cpu().numpy()
        for r in range(w["Q"].shape[0]):
            ref = O.probes(oi, w["Q"][r], qp, "gap")
            assert sorted(g[r].tolist()) == sorted(ref.tolist()), (qp, r)
    qp = 4 * w["L"]
    ids, sc = F().fpp_query(h, Qd, 10, qp, probe_score="gap")
    oids, osc, _ = O.query(oi, w["Q"], 10, qp, "gap")
    swaps = check_topk(w["X"], w["Q"], ids.cpu().numpy(), sc.cpu().numpy(), oids, osc)
    assert swaps <= swap_budget(ids.numel()), swaps


@pytest.mark.parametrize("name", list(CONFIGS))
@pytest.mark.parametrize("k", [1, 10, 100])
def test_query_fp32_matches_oracle(name, k):
    w, oi, h, Xd, Qd = built(name)
    qp = 8 * w["L"]
    ids, sc, st = F().fpp_query(h, Qd, k, qp, stats=True)
    oids, osc, ost = O.query(oi, w["Q"], k, qp)
    np.testing.assert_array_equal(st.cpu().numpy(), ost)
    swaps = check_topk(w["X"], w["Q"], ids.cpu().numpy(), sc.cpu().numpy(), oids, osc)
    assert swaps <= swap_budget(ids.numel()), swaps


@pytest.mark.parametrize("qp", [2000, 10 ** 6])
def test_query_many_candidates_uses_bitmap_dedup(qp):
    """More distinct candidates than the LDS id set holds: dedup moves to the device bitmap."""
    w, oi, h, Xd, Qd = built("l2_clustered")
    ids, sc, st = F().fpp_query(h, Qd, 100, qp, stats=True)
    oids, osc, ost = O.query(oi, w["Q"], 100, qp)
    st = st.cpu().numpy()
    np.testing.assert_array_equal(st, ost)
    assert st[:, 2].max() > 3072
    swaps = check_topk(w["X"], w["Q"], ids.cpu().numpy(), sc.cpu().numpy(), oids, osc)
    assert swaps <= swap_budget(ids.numel()), swaps
    # a second call reuses the (cleared) bitmaps
    ids2, sc2 = F().fpp_query(h, Qd, 100, qp)
    assert torch.equal(ids, ids2) and torch.equal(sc, sc2)


@pytest.mark.parametrize("name,qp,bits", [("c1_gauss_10k_d64", 8, 8), ("l2_clustered", 16, 8),
                                           ("l2_clustered", 40, 7), ("pad_d100_D16", 4, 5),
                                           ("manyL_d24_L40", 2, 5), ("odd_d30_D32", 4, 5)])
def test_partitioned_dedup_matches_oracle(name, qp, bits):
    """Queries deduplicated by id range (forced for every query whose probed entries fit the
    workgroup's buffer of n / 32 ids, in ranges of 2^bits ids) give the oracle's candidate counts
    and top-k (Section 4: each candidate is scored once), and the same ids and scores as the
    on-chip set, on the FP32 and the BF16 + rerank paths."""
    w, oi, h, Xd, Qd = built(name)
    n = w["X"].shape[0]
    bm_words = ((n + 31) // 32 + 3) & ~3
    ref = {st: F().fpp_query(h, Qd, 10, qp, store=st) for st in ("fp32", "bf16")}
    F().fpp_debug_set_partition_threshold(h, 0, bits)
    try:
        ids, sc, st = F().fpp_query(h, Qd, 10, qp, stats=True)
        low = F().fpp_query(h, Qd, 10, qp, store="bf16")
    finally:
        F().fpp_debug_set_partition_threshold(h, -1, -1)
    st = st.cpu().numpy()
    assert ((st[:, 1] > 0) & (st[:, 1] <= bm_words)).sum() >= 3   # queries that took the path
    oids, osc, ost = O.query(oi, w["Q"], 10, qp)
    np.testing.assert_array_equal(st, ost)
    swaps = check_topk(w["X"], w["Q"], ids.cpu().numpy(), sc.cpu().numpy(), oids, osc)
    assert swaps <= swap_budget(ids.numel()), swaps
    assert torch.equal(ids, ref["fp32"][0]) and torch.equal(sc, ref["fp32"][1])
    assert torch.equal(low[0], ref["bf16"][0]) and torch.equal(low[1], ref["bf16"][1])


def test_concurrent_queries_on_two_streams_share_the_bitmaps():
    """Calls on two streams in flight at once (one spilling into the overflow bitmaps, one not)
    each equal the same call made alone: the index's bitmaps and work counters are handed over
    between the calls."""
    w, oi, h, Xd, Qd = built("l2_clustered")
    ref_a = F().fpp_query(h, Qd, 100, 2000)
    ref_b = F().fpp_query(h, Qd.flip(0).contiguous(), 10, 24, store="bf16")
    torch.cuda.synchronize()
    sa, sb = torch.cuda.Stream(), torch.cuda.Stream()
    Qb = Qd.flip(0).contiguous()
    torch.cuda.synchronize()
    outs = []
    for _ in range(3):
        with torch.cuda.stream(sa):
            ra = F().fpp_query(h, Qd, 100, 2000, stream=sa)
        with torch.cuda.stream(sb):
            rb = F().fpp_query(h, Qb, 10, 24, store="bf16", stream=sb)
        outs.append((ra, rb))
    torch.cuda.synchronize()
    for ra, rb in outs:
        assert torch.equal(ra[0], ref_a[0]) and torch.equal(ra[1], ref_a[1])
        assert torch.equal(rb[0], ref_b[0]) and torch.equal(rb[1], ref_b[1])


def test_calls_on_two_streams_take_separate_bitmaps():
    """A call issued on one stream while another call on the same index is still running takes a
    second set of overflow bitmaps instead of waiting for the first call (the index hands each
    in-flight call its own set); both results equal the calls made alone."""
    X, Q = synthdata.clustered_sphere(20_000, 128, 40, 50, 0.3, seed=7)
    Xd, Qd = torch.from_numpy(X).cuda(), torch.from_numpy(Q).cuda()
    h = F().fpp_build_index(Xd, 6, 32, 0.3, 3, SEED, l=2)
    try:
        Qbig = Qd.repeat(100, 1).contiguous()   # 4,000 queries with 2,000 probes each: a long call
        ref_a = F().fpp_query(h, Qbig, 10, 2000)
        torch.cuda.synchronize()
        ref_b = F().fpp_query(h, Qd, 10, 48)
        torch.cuda.synchronize()
        assert F().fpp_index_get_info(h)["overflow_sets"] == 1   # calls one after another share one
        sa, sb = torch.cuda.Stream(), torch.cuda.Stream()
        with torch.cuda.stream(sa):
            ra = F().fpp_query(h, Qbig, 10, 2000, stream=sa)
        with torch.cuda.stream(sb):
            rb = F().fpp_query(h, Qd, 10, 48, stream=sb)
        torch.cuda.synchronize()
        assert F().fpp_index_get_info(h)["overflow_sets"] == 2
        assert torch.equal(ra[0], ref_a[0]) and torch.equal(ra[1], ref_a[1])
        assert torch.equal(rb[0], ref_b[0]) and torch.equal(rb[1], ref_b[1])
    finally:
        F().fpp_free_index(h)


def test_query_c1_published_qprobes():
    """The small workload as specified: k = 10, 4 probes per table (40 in total), and the
    literal total of 4."""
    w, oi, h, Xd, Qd = built("c1_gauss_10k_d64")
    for qp in (40, 4):
        ids, sc = F().fpp_query(h, Qd, 10, qp)
        oids, osc, _ = O.query(oi, w["Q"], 10, qp)
        swaps = check_topk(w["X"], w["Q"], ids.cpu().numpy(), sc.cpu().numpy(), oids, osc)
        assert swaps <= swap_budget(ids.numel()), swaps


# ----------------------------------------------------------------------------------------------
def test_mixed_batch_equals_single_queries():
    w, oi, h, Xd, Qd = built("l2_clustered")
    m = Qd.shape[0]
    rng = np.random.default_rng(0)
    ks = rng.choice([1, 10, 100], size=m)
    qps = rng.choice([20, 50, 200], size=m) * w["L"] // 4
    bi, bs = F().fpp_query_batch(h, Qd, ks, qps)
    bi, bs = bi.cpu().numpy(), bs.cpu().numpy()
    off = 0
    for r in range(m):
        si, ss = F().fpp_query(h, Qd[r:r + 1].contiguous(), int(ks[r]), int(qps[r]))
        np.testing.assert_array_equal(bi[off:off + ks[r]], si.cpu().numpy()[0])
        np.testing.assert_array_equal(bs[off:off + ks[r]].view(np.uint32), ss.cpu().numpy()[0].view(np.uint32))
        off += ks[r]


def test_determinism_rebuild_and_requery():
    w, oi, h, Xd, Qd = built("l2_clustered")
    h2 = F().fpp_build_index(Xd, w["L"], w["D"], w["alpha"], w["iProbes"], SEED, l=w["l"], tables_per_pass=1)
    try:
        for t in range(w["L"]):
            a = F().fpp_debug_export_table(h, t)
            b = F().fpp_debug_export_table(h2, t)
            np.testing.assert_array_equal(a[0], b[0])
            np.testing.assert_array_equal(a[1], b[1])
        r1 = F().fpp_query(h, Qd, 10, 100)
        r2 = F().fpp_query(h2, Qd, 10, 100)
        s = torch.cuda.Stream()
        with torch.cuda.stream(s):
            r3 = F().fpp_query(h, Qd, 10, 100)
        s.synchronize()
        for r in (r2, r3):
            assert torch.equal(r1[0], r[0]) and torch.equal(r1[1], r[1])
    finally:
        F().fpp_free_index(h2)


def test_chunked_queries_equal_one_chunk():
    """Many queries (more than one persistent pass per block) give the per-query results."""
    w, oi, h, Xd, Qd = built("wideD_d20_D64")
    Qbig = Qd.repeat(40, 1).contiguous()
    ids, sc = F().fpp_query(h, Qbig, 10, 30)
    ref_i, ref_s = F().fpp_query(h, Qd, 10, 30)
    m = Qd.shape[0]
    for rep in range(40):
        assert torch.equal(ids[rep * m:(rep + 1) * m], ref_i)
        assert torch.equal(sc[rep * m:(rep + 1) * m], ref_s)


# ----------------------------------------------------------------------------------------------
# edge cases
def _small_index(X, L, D, alpha, iProbes, l, seed=3):
    Xd = torch.from_numpy(np.ascontiguousarray(X, dtype=np.float32)).cuda()
    return Xd, F().fpp_build_index(Xd, L, D, alpha, iProbes, seed, l=l)


def test_padding_when_fewer_candidates_than_k():
    X, Q = synthdata.clustered_sphere(500, 16, 5, 5, 0.4, seed=1)
    Xd, h = _small_index(X, 2, 8, 0.2, 1, 2)
    try:
        oi = O.build_index(X, 2, 8, 0.2, 1, 3, l=2)
        Qd = torch.from_numpy(Q).cuda()
        ids, sc = F().fpp_query(h, Qd, 512, 1)
        oids, osc, _ = O.query(oi, Q, 512, 1)
        check_topk(X, Q, ids.cpu().numpy(), sc.cpu().numpy(), oids, osc)
        assert (ids.cpu().numpy() == -1).any()
    finally:
        F().fpp_free_index(h)


def test_n_smaller_than_k_and_full_probing():
    X, Q = synthdata.clustered_sphere(5, 8, 3, 2, 0.5, seed=2)
    Xd, h = _small_index(X, 3, 4, 1.0, 1, 2)
    try:
        oi = O.build_index(X, 3, 4, 1.0, 1, 3, l=2)
        Qd = torch.from_numpy(Q).cuda()
        ids, sc = F().fpp_query(h, Qd, 10, 10 ** 6)
        oids, osc, _ = O.query(oi, Q, 10, 10 ** 6)
        check_topk(X, Q, ids.cpu().numpy(), sc.cpu().numpy(), oids, osc)
    finally:
        F().fpp_free_index(h)


def test_duplicate_points_and_zero_query():
    X, Q = synthdata.clustered_sphere(800, 32, 6, 4, 0.3, seed=3)
    X[10] = X[5]
    X[11] = X[5]
    Q[0] = X[5]
    Q[1] = 0.0
    Xd, h = _small_index(X, 4, 16, 0.5, 2, 2)
    try:
        oi = O.build_index(X, 4, 16, 0.5, 2, 3, l=2)
        for t in range(4):
            off, ids = F().fpp_debug_export_table(h, t)
            np.testing.assert_array_equal(ids, oi.ids[t])
        Qd = torch.from_numpy(Q).cuda()
        ids, sc = F().fpp_query(h, Qd, 10, 64)
        oids, osc, _ = O.query(oi, Q, 10, 64)
        check_topk(X, Q, ids.cpu().numpy(), sc.cpu().numpy(), oids, osc)
        got = ids.cpu().numpy()[0][:3].tolist()
        assert got == [5, 10, 11] or oids[0][:3].tolist() != [5, 10, 11]
        np.testing.assert_array_equal(ids.cpu().numpy()[0], oids[0])
    finally:
        F().fpp_free_index(h)


def test_huge_buckets_beyond_lds_sort():
    """Buckets of more than 8192 records (many equal points) are ranked by counting."""
    rng = np.random.default_rng(5)
    base = rng.standard_normal((3, 16))
    base /= np.linalg.norm(base, axis=1, keepdims=True)
    X = base[rng.integers(0, 3, size=30_000)].astype(np.float32)
    X[::7] += np.float32(1e-3)          # some distinct keys among the equal ones
    for l, D, ip in ((1, 8, 1), (2, 4, 2)):
        Xd, h = _small_index(X, 2, D, 0.4, ip, l)
        try:
            oi = O.build_index(X, 2, D, 0.4, ip, 3, l=l)
            assert max(int(np.max(np.diff(o))) for o in oi.offsets) > 2000
            for t in range(2):
                off, ids = F().fpp_debug_export_table(h, t)
                np.testing.assert_array_equal(off, oi.offsets[t])
                np.testing.assert_array_equal(ids, oi.ids[t])
        finally:
            F().fpp_free_index(h)


def test_tiny_d1_D2_L1():
    X = np.where(np.arange(50) % 2 == 0, 1.0, -1.0).astype(np.float32)[:, None]
    Q = np.array([[1.0], [-1.0]], np.float32)
    Xd, h = _small_index(X, 1, 2, 1.0, 1, 1)
    try:
        oi = O.build_index(X, 1, 2, 1.0, 1, 3, l=1)
        off, ids = F().fpp_debug_export_table(h, 0)
        np.testing.assert_array_equal(off, oi.offsets[0])
        np.testing.assert_array_equal(ids, oi.ids[0])
        Qd = torch.from_numpy(Q).cuda()
        gi, gs = F().fpp_query(h, Qd, 5, 2)
        oids, osc, _ = O.query(oi, Q, 5, 2)
        np.testing.assert_array_equal(gi.cpu().numpy(), oids)
    finally:
        F().fpp_free_index(h)


def test_empty_query_batch_and_errors():
    w, oi, h, Xd, Qd = built("l2_clustered")
    ids, sc = F().fpp_query(h, Qd[:0], 10, 10)
    assert ids.shape == (0, 10)
    with pytest.raises(F().FppError):
        F().fpp_query(h, Qd, 0, 10)
    with pytest.raises(F().FppError):
        F().fpp_query(h, Qd, 600, 10)
    with pytest.raises(F().FppError):
        F().fpp_query(h, Qd, 10, 0)
    h1 = F().fpp_build_index(Xd, 2, 16, 0.5, 1, 5)
    try:
        with pytest.raises(F().FppError) as e:
            F().fpp_query(h1, Qd, 10, 10, store="bf16")
        assert e.value.code == F().FPP_ESTATE
    finally:
        F().fpp_free_index(h1)


# ----------------------------------------------------------------------------------------------
# limit scaling, centering and the global-threshold filter
HEUR = {
    "kappa5": dict(kappa=5),
    "center": dict(center=True),
    "center_kappa3": dict(center=True, kappa=3),
    "lsf_derived_t": dict(filter="threshold"),
    "lsf_given_t": dict(filter="threshold", threshold=0.9),
    "lsf_center_l1": dict(filter="threshold", center=True, l=1),
}


@pytest.mark.parametrize("name", list(HEUR))
def test_heuristic_builds_bit_exact(name):
    opts = dict(HEUR[name])
    l = opts.pop("l", 2)
    X, Q = synthdata.clustered_sphere(6_000, 64, 30, 12, 0.4, seed=31)
    X = (X + np.float32(0.15)).astype(np.float32)          # off-centre, so that c matters
    L, D, alpha, K = 3, 16, 0.3, 3
    oi = O.build_index(X, L, D, alpha, K, SEED, l=l, **opts)
    Xd = torch.from_numpy(X).cuda()
    h = F().fpp_build_index(Xd, L, D, alpha, K, SEED, l=l, **opts)
    try:
        inf = F().fpp_index_get_info(h)
        assert inf["kappa"] == (0 if opts.get("filter") == "threshold" else opts.get("kappa", 0))
        assert inf["centered"] == int(opts.get("center", False))
        if opts.get("filter") == "threshold":
            assert np.float32(inf["threshold"]) == oi.threshold
        c = F().fpp_debug_center(h)
        np.testing.assert_array_equal(c, oi.center if oi.center is not None else np.zeros(64, np.float32))
        for t in range(L):
            off, ids = F().fpp_debug_export_table(h, t)
            np.testing.assert_array_equal(off, oi.offsets[t])
            np.testing.assert_array_equal(ids, oi.ids[t])
        if opts.get("center") and opts.get("filter") != "threshold":
            b, k = F().fpp_debug_build_records(h, 1)
            lists = [O.hash_lists((X - oi.center).astype(np.float32), oi.signs[1, f], D) for f in range(l)]
            ob, ok = O.top_pairs(lists, D, K)
            np.testing.assert_array_equal(b.cpu().numpy().astype(np.int64), ob)
        Qd = torch.from_numpy(Q).cuda()
        ids, sc = F().fpp_query(h, Qd, 10, 8 * L)
        oids, osc, _ = O.query(oi, Q, 10, 8 * L)
        swaps = check_topk(X, Q, ids.cpu().numpy(), sc.cpu().numpy(), oids, osc)
        assert swaps <= swap_budget(ids.numel()), swaps
    finally:
        F().fpp_free_index(h)


# ----------------------------------------------------------------------------------------------
# precision stores
@pytest.mark.parametrize("name", ["l2_clustered", "p512_d300_D256", "c1_gauss_10k_d64", "max_d1024_D1024_ip16"])
def test_stores_bit_exact(name):
    w, oi, h, Xd, Qd = built(name)
    b, _ = F().fpp_debug_export_store(h, "bf16")
    np.testing.assert_array_equal(b.cpu().numpy().view(np.uint16), O.bf16_bits(w["X"]))
    c, s = F().fpp_debug_export_store(h, "fp8")
    oc, os_ = O.quantize_fp8_rows(w["X"])
    np.testing.assert_array_equal(s.cpu().numpy().view(np.uint32), os_.view(np.uint32))
    np.testing.assert_array_equal(c.cpu().numpy(), oc)


@pytest.mark.parametrize("name", ["l2_clustered", "p512_d300_D256", "max_d1024_D1024_ip16"])
@pytest.mark.parametrize("store", ["bf16", "fp8"])
def test_query_low_precision_with_rerank(name, store):
    w, oi, h, Xd, Qd = built(name)
    k, qp = 10, 8 * w["L"]
    ids, sc = F().fpp_query(h, Qd, k, qp, store=store)
    oids, osc, _ = O.query_reranked(oi, w["Q"], k, qp, R=100, storage=store)
    swaps = check_topk(w["X"], w["Q"], ids.cpu().numpy(), sc.cpu().numpy(), oids, osc)
    assert swaps <= swap_budget(ids.numel()), swaps
    # rerank scores equal the exact FP32 path's scores for the same ids
    fi, fs = F().fpp_query(h, Qd, k, qp)
    same = (ids == fi).all(dim=1)
    assert torch.equal(sc[same], fs[same])


@pytest.mark.parametrize("name", ["l2_clustered", "p512_d300_D256"])
@pytest.mark.parametrize("store", ["bf16", "fp8"])
def test_query_low_precision_without_rerank(name, store):
    """rerank_R = -1: the top-k of the approximate pass itself, scored on the dequantised store.

    Scores are checked against float64 dot products with the dequantised rows (the FP32
    accumulation bound), ids against exact search over the same candidates on that store."""
    w, oi, h, Xd, Qd = built(name)
    k, qp = 10, 8 * w["L"]
    deq = O.dequantized_store(w["X"], store)
    ids, sc = F().fpp_query(h, Qd, k, qp, store=store, rerank_R=-1)
    gi, gs = ids.cpu().numpy(), sc.cpu().numpy()
    m = w["Q"].shape[0]
    oids = np.empty((m, k), dtype=np.int64)
    osc = np.empty((m, k))
    for r in range(m):
        cand = O.candidates(oi, O.probes(oi, w["Q"][r], qp))
        oids[r], osc[r] = O.topk_order(deq[cand] @ w["Q"][r].astype(np.float64), cand, k)
    swaps = check_topk(deq, w["Q"], gi, gs, oids, osc)
    assert swaps <= swap_budget(gi.size), swaps


@pytest.mark.parametrize("store", ["fp32", "bf16", "fp8"])
def test_maximum_sizes_k512_rerank512(store):
    """k = 512 with a rerank of R = 512 at d = 1024, the largest k, R and d the boundary takes:
    the FP32 top-512 (and the reranked low-precision top-512) against the oracle's."""
    w, oi, h, Xd, Qd = built("max_d1024_D1024_ip16")
    k, qp = 512, 20_000   # about 600 candidates per query
    if store == "fp32":
        ids, sc, st = F().fpp_query(h, Qd, k, qp, stats=True)
        oids, osc, ost = O.query(oi, w["Q"], k, qp)
        np.testing.assert_array_equal(st.cpu().numpy(), ost)
    else:
        ids, sc = F().fpp_query(h, Qd, k, qp, store=store, rerank_R=512)
        oids, osc, _ = O.query_reranked(oi, w["Q"], k, qp, R=512, storage=store)
    gi = ids.cpu().numpy()
    assert (gi >= 0).sum() > 0.9 * gi.size   # most rows hold 512 candidates
    swaps = check_topk(w["X"], w["Q"], gi, sc.cpu().numpy(), oids, osc)
    assert swaps <= swap_budget(ids.numel()), swaps


def _near_duplicate_sphere(groups, per, d, m, seed):
    """Groups of near-duplicate unit vectors (8e-3 per coordinate around a random unit direction)
    and queries near some of the directions: a group's scores spread over about 2.6e-3, less than
    twice the rerank's bound (about 3.9e-3 at d = 64), so the cut's boundary falls among them,
    while their gaps (at least about 4e-7 here) stay above float32 rounding."""
    rng = np.random.default_rng(seed)
    base = rng.standard_normal((groups, d))
    base /= np.linalg.norm(base, axis=1, keepdims=True)
    X = np.repeat(base, per, axis=0) + 8e-3 * rng.standard_normal((groups * per, d))
    X /= np.linalg.norm(X, axis=1, keepdims=True)
    Q = base[:m] + 1e-2 * rng.standard_normal((m, d))
    Q /= np.linalg.norm(Q, axis=1, keepdims=True)
    return X.astype(np.float32), Q.astype(np.float32)


@pytest.mark.parametrize("name", ["l2_clustered", "p512_d300_D256", "fused_d128_D128", "near_duplicates"])
def test_rerank_cut_changes_nothing(name):
    """BF16 + rerank with the cut (only the rows that can still reach the top k are rescored, and
    the gather drops the others as it scores) against rescoring every short-listed row: equal ids
    and scores, bit for bit, for several k and short-list lengths; and equal to the oracle."""
    own = name == "near_duplicates"
    if own:
        X, Q = _near_duplicate_sphere(200, 20, 64, 30, seed=5)
        Xd = torch.from_numpy(X).cuda()
        h = F().fpp_build_index(Xd, 4, 64, 0.5, 3, SEED, l=2, stores=("bf16",))
        Qd = torch.from_numpy(Q).cuda()
        L = 4
    else:
        w, oi, h, Xd, Qd = built(name)
        X, Q, L = w["X"], w["Q"], w["L"]
    try:
        qp = 8 * L
        for k, R in ((1, 0), (10, 0), (10, 30), (50, 0), (50, 150)):
            F().fpp_debug_set_rerank_cut(h, True)
            ids_c, sc_c = F().fpp_query(h, Qd, k, qp, store="bf16", rerank_R=R)
            F().fpp_debug_set_rerank_cut(h, False)
            ids_f, sc_f = F().fpp_query(h, Qd, k, qp, store="bf16", rerank_R=R)
            assert torch.equal(ids_c, ids_f), (k, R)
            assert torch.equal(sc_c.view(torch.int32), sc_f.view(torch.int32)), (k, R)
        if own:
            oi = O.build_index(X, 4, 64, 0.5, 3, SEED, l=2)
        F().fpp_debug_set_rerank_cut(h, True)
        ids, sc = F().fpp_query(h, Qd, 10, qp, store="bf16")
        oids, osc, _ = O.query_reranked(oi, Q, 10, qp, R=100, storage="bf16")
        swaps = check_topk(X, Q, ids.cpu().numpy(), sc.cpu().numpy(), oids, osc)
        assert swaps <= swap_budget(ids.numel()), swaps
    finally:
        F().fpp_debug_set_rerank_cut(h, True)
        if own:
            F().fpp_free_index(h)


def test_rerank_of_exactly_k_is_a_reorder_with_exact_scores():
    """With R = k the rerank reorders the approximate top-k; its scores are exact FP32 dot
    products of the original rows (float64 within the FP32 accumulation bound)."""
    w, oi, h, Xd, Qd = built("l2_clustered")
    d = w["X"].shape[1]
    for store in ("bf16", "fp8"):
        ai, _ = F().fpp_query(h, Qd, 100, 8 * w["L"], store=store, rerank_R=-1)
        ids, sc = F().fpp_query(h, Qd, 100, 8 * w["L"], store=store, rerank_R=100)
        gi, ga, gs = ids.cpu().numpy().astype(np.int64), ai.cpu().numpy(), sc.cpu().numpy()
        for r in range(gi.shape[0]):
            assert sorted(gi[r].tolist()) == sorted(ga[r].tolist())
            v = gi[r][gi[r] >= 0]
            x64 = w["X"][v].astype(np.float64)
            q64 = w["Q"][r].astype(np.float64)
            s64 = x64 @ q64
            tol = score_tol(s64, np.abs(x64 * q64).sum(1))
            assert np.all(np.abs(gs[r][: len(v)] - s64) <= tol)
            assert np.all(np.diff(gs[r][: len(v)]) <= 0)


# ----------------------------------------------------------------------------------------------
# SimHash pre-scoring
@pytest.mark.parametrize("D,nf,l", [(32, 8, 2), (128, 2, 2), (16, 6, 1)])
def test_simhash_store_and_queries(D, nf, l):
    X, Q = synthdata.clustered_sphere(5_000, 64, 25, 10, 0.4, seed=33)
    L = max(4, -(-nf // l))
    oi = O.build_index(X, L, D, 0.4, 3, SEED, l=l)
    Xd, Qd = torch.from_numpy(X).cuda(), torch.from_numpy(Q).cuda()
    h = F().fpp_build_index(Xd, L, D, 0.4, 3, SEED, l=l, stores=("simhash",), simhash_functions=nf)
    try:
        assert F().fpp_index_get_info(h)["simhash_bits"] == nf * D
        bits = O.simhash_bits(X, oi.signs, D, nf)
        codes, _ = F().fpp_debug_export_store(h, "simhash")
        np.testing.assert_array_equal(codes.cpu().numpy().view(np.uint32), O.simhash_words(bits))
        qp = 6 * L
        # the approximate pass itself: integer scores, ordered (score desc, id asc) -> exact
        ai, asc = F().fpp_query(h, Qd, 10, qp, store="simhash", rerank_R=-1)
        qbits = O.simhash_bits(Q, oi.signs, D, nf)
        for r in range(Q.shape[0]):
            cand = O.candidates(oi, O.probes(oi, Q[r], qp))
            ri, rs = O.topk_order(O.simhash_score(bits[cand], qbits[r]), cand, 10)
            assert np.array_equal(ai.cpu().numpy()[r], ri.astype(np.int32)), r
            assert np.array_equal(asc.cpu().numpy()[r], rs.astype(np.float32)), r
        # with the FP32 rerank of a short list of 100
        ids, sc = F().fpp_query(h, Qd, 10, qp, store="simhash", rerank_R=100)
        oids, osc, _ = O.query_reranked(oi, Q, 10, qp, R=100, storage="simhash", simhash_functions=nf)
        swaps = check_topk(X, Q, ids.cpu().numpy(), sc.cpu().numpy(), oids, osc)
        assert swaps <= swap_budget(ids.numel()), swaps
    finally:
        F().fpp_free_index(h)


# ----------------------------------------------------------------------------------------------
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _golden(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def _compare_fullsize(g, w, h, Qd, tables=True):
    """Tables, probe sets, candidate counts and top-k of the sampled queries against the oracle's
    stored values; every query call covers the whole batch (the benchmark's launch shape)."""
    rows = np.asarray(g["queries"], dtype=np.int64)
    if tables:
        print(f"{g['workload']}: {g['L']} tables against the oracle", flush=True)
        sizes = F().fpp_index_table_sizes(h)
        for t, rec in enumerate(g["tables"]):
            off, ids = F().fpp_debug_export_table(h, t)
            assert sizes[t] == rec["size"] and int(np.max(np.diff(off))) == rec["max_bucket"], t
            assert table_digest(off, ids) == rec["sha256"], t
    Qs = Qd[torch.from_numpy(rows).cuda()].contiguous()
    for qp, ref in g["fp32"].items():
        print(f"{g['workload']}: FP32 path, qProbes {qp}", flush=True)
        gi, gs, st = F().fpp_query(h, Qd, 10, int(qp), stats=True)
        gi, gs, st = gi.cpu().numpy()[rows], gs.cpu().numpy()[rows], st.cpu().numpy()[rows]
        np.testing.assert_array_equal(st, np.asarray(ref["stats"]))
        swaps = check_topk(w.X, w.Q[rows], gi, gs, np.asarray(ref["ids"]), np.asarray(ref["scores"]),
                           label=f"{g['workload']} fp32 qProbes={qp}")
        assert swaps <= swap_budget(gi.size), swaps
        if "probe_sha256" in ref:
            pr = F().fpp_debug_probes(h, Qs, int(qp)).cpu().numpy()
            assert [probe_digest(p) for p in pr] == ref["probe_sha256"]
    for store, ref in g["rerank"].items():
        qp = int(ref["qProbes"])
        print(f"{g['workload']}: {store} + rerank of {ref['R']}, qProbes {qp}", flush=True)
        gi, gs = F().fpp_query(h, Qd, 10, qp, store=store, rerank_R=int(ref["R"]))
        gi, gs = gi.cpu().numpy()[rows], gs.cpu().numpy()[rows]
        swaps = check_topk(w.X, w.Q[rows], gi, gs, np.asarray(ref["ids"]), np.asarray(ref["scores"]),
                           label=f"{g['workload']} {store}+rerank qProbes={qp}")
        assert swaps <= swap_budget(gi.size), swaps


@pytest.mark.timeout(600)
def test_full_size_c2_against_oracle():
    """The headline index (n = 1M, d = 128, L = 100, D = 128, l = 2, alpha = 0.3, iProbes = 3)
    against the oracle's own index and answers (stored by tests/golden/make_fullsize_oracle.py):
    all 100 tables bit-exact, and for 200 queries spread over the 10,000-query batch the probe
    sets (27 in total, the benchmark's operating point), the candidate counts and the FP32
    top-10 at 27 and 50 probes and at 50 per table, and the BF16 and FP8 paths with the FP32
    rerank of 100 at 27 probes."""
    g = _golden("c2_full_oracle.json")
    w = synthdata.workload("c2_cluster_1m_d128")
    assert (g["n"], g["d"], g["L"], g["D"]) == (w.X.shape[0], w.X.shape[1], w.L, w.D)
    Xd = torch.from_numpy(w.X).cuda()
    h = F().fpp_build_index(Xd, w.L, w.D, w.alpha, w.iProbes, g["seed"], l=w.l, stores=("bf16", "fp8"))
    try:
        np.testing.assert_array_equal(F().fpp_debug_signs(h), O.rotation_signs(g["seed"], w.L, w.l, 128))
        _compare_fullsize(g, w, h, torch.from_numpy(w.Q).cuda())
    finally:
        F().fpp_free_index(h)


@pytest.mark.timeout(900)
def test_c5_shape_against_oracle():
    """The large workload's data and table shape (n = 10M, d = 96 zero-padded to P = 256, D = 256,
    l = 2, alpha = 0.1, iProbes = 2) with 4 of its 64 tables: every table bit-exact against the
    oracle's, and for 200 of the 100,000 queries (one launch) the probe sets at 100 probes per
    table, the candidate counts, the FP32 top-10 and the FP8 path with the FP32 rerank of 100."""
    g = _golden("c5_shape_oracle.json")
    print("c5 shape: drawing 10M x 96", flush=True)
    w = synthdata.workload("c5_cluster_10m_d96")
    assert (g["n"], g["d"], g["D"]) == (w.X.shape[0], w.X.shape[1], w.D)
    Xd = torch.from_numpy(w.X).cuda()
    h = F().fpp_build_index(Xd, g["L"], w.D, w.alpha, w.iProbes, g["seed"], l=w.l, stores=("fp8",))
    try:
        Qd = torch.from_numpy(w.Q).cuda()
        _compare_fullsize(g, w, h, Qd)
        # every query deduplicated by id range (39 ranges of 2^18 ids, two probe chunks)
        print("c5 shape: dedup by id range", flush=True)
        F().fpp_debug_set_partition_threshold(h, 0, -1)
        _compare_fullsize(g, w, h, Qd, tables=False)
    finally:
        F().fpp_free_index(h)
        del Xd


@pytest.mark.timeout(600)
def test_full_size_precision_form_sampled():
    """n = 1M, d = 300 (P = 512), L = 128, D = 256, l = 2, alpha = 0.2, iProbes = 3 with the BF16
    and FP8 stores, 10,000 queries in one launch: sampled rows of both stores bit-exact, sampled
    probe sets bit-exact, and the sampled queries' FP32 top-k and unreranked BF16 / FP8 top-k equal
    to exact search (on the exact or the dequantised rows) over the candidates their probes select,
    at 101 probes (fused hash-and-select kernel) and 200 (list kernels)."""
    w = synthdata.workload("c3_cluster_1m_d300")
    Xd = torch.from_numpy(w.X).cuda()
    h = F().fpp_build_index(Xd, w.L, w.D, w.alpha, w.iProbes, 42, l=w.l, stores=("bf16", "fp8"))
    try:
        S = O.rotation_signs(42, w.L, w.l, 512)
        np.testing.assert_array_equal(F().fpp_debug_signs(h), S)
        rows = np.array([0, 1, 777_777, w.X.shape[0] - 1])
        b, _ = F().fpp_debug_export_store(h, "bf16")
        np.testing.assert_array_equal(b.cpu().numpy().view(np.uint16)[rows], O.bf16_bits(w.X[rows]))
        c, sc8 = F().fpp_debug_export_store(h, "fp8")
        oc, os_ = O.quantize_fp8_rows(w.X[rows])
        np.testing.assert_array_equal(c.cpu().numpy()[rows], oc)
        np.testing.assert_array_equal(sc8.cpu().numpy()[rows].view(np.uint32), os_.view(np.uint32))
        del b, c, sc8
        Qd = torch.from_numpy(w.Q).cuda()
        # 101 probes (at most one per table: the fused hash-and-select kernel) and 200 (the list
        # kernels)
        for qp in (101, 200):
            shell = O.Index(X=w.X, L=w.L, D=w.D, l=w.l, P=512, alpha=w.alpha, iProbes=w.iProbes, seed=42, signs=S)
            NB = O.n_buckets(w.D, w.l)
            print(f"full-size c3: qProbes {qp}: FP32 and approximate passes", flush=True)
            gi, gs = F().fpp_query(h, Qd, 10, qp)
            appr = {st: F().fpp_query(h, Qd, 10, qp, store=st, rerank_R=-1) for st in ("bf16", "fp8")}
            gi, gs = gi.cpu().numpy(), gs.cpu().numpy()
            appr = {st: (a.cpu().numpy(), b.cpu().numpy()) for st, (a, b) in appr.items()}
            tables = {}

            def local(ids, cand):      # candidate ids -> rows of the candidate submatrix
                ids = ids.astype(np.int64)
                pos = np.searchsorted(cand, np.maximum(ids, 0))
                ok = ids >= 0
                assert np.all(cand[np.minimum(pos[ok], len(cand) - 1)] == ids[ok])
                return np.where(ok, pos, -1)

            for r in (0, 4_321, w.Q.shape[0] - 1):
                print(f"full-size c3: qProbes {qp}, query {r}", flush=True)
                pr = O.probes(shell, w.Q[r], qp)
                gp = F().fpp_debug_probes(h, Qd[r:r + 1].contiguous(), qp).cpu().numpy()[0]
                assert sorted(gp.tolist()) == sorted(pr.tolist())
                cand = []
                for p in pr:
                    t, bk = divmod(int(p), NB)
                    if t not in tables:
                        tables[t] = F().fpp_debug_export_table(h, t)
                    off, ids = tables[t]
                    cand.append(ids[off[bk]:off[bk + 1]])
                cand = np.unique(np.concatenate(cand).astype(np.int64))
                pos = np.arange(len(cand))
                q = w.Q[r:r + 1]
                Xc = w.X[cand]
                ri, rs = O.topk_order(Xc.astype(np.float64) @ q[0].astype(np.float64), pos, 10)
                check_topk(Xc, q, local(gi[r:r + 1], cand), gs[r:r + 1], ri[None], rs[None], 10, 300)
                for st, (ai, asc) in appr.items():
                    dq = O.dequantized_store(Xc, st)
                    bi, bs = O.topk_order(dq @ q[0].astype(np.float64), pos, 10)
                    check_topk(dq, q, local(ai[r:r + 1], cand), asc[r:r + 1], bi[None], bs[None], 10, 300, st)
    finally:
        F().fpp_free_index(h)
