"""Pins of the CPU oracle against facts that do not come from the oracle itself.

Each test names what pins it: a closed form (Sylvester Hadamard matrices), the
published SplitMix64 outputs, an invariant the paper states (Algorithm 1:
iProbes buckets per point, alpha*n points per table; Section 4: Falconn is
Falconn++ with alpha = 1 and iProbes = 1), a special case (full probing reaches every
sign-consistent point), a library routine (scipy's Hadamard, torch's bf16 / fp8 casts)
or brute-force enumeration on tiny inputs written with Python loops.
"""
import math
import os

import numpy as np
import pytest
import scipy.linalg

from oracle import falconn as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ------------------------------------------------------------------ signs
def test_splitmix64_published_outputs():
    vals = [int(l) for l in open(os.path.join(GOLDEN, "splitmix64_seed1234567.txt"))
            if l.strip() and not l.startswith("#")]
    got = [int(v) for v in O.splitmix64_at(1234567, np.arange(5))]
    assert got == vals


def _splitmix64_stepped(seed, count):
    """The published generator as a stateful stream (splitmix64.c, next()): advance the state by
    the golden-ratio increment, then mix; a loop over Python integers, independent of the
    oracle's closed form for output c."""
    mask = (1 << 64) - 1
    state = seed & mask
    out = []
    for _ in range(count):
        state = (state + 0x9E3779B97F4A7C15) & mask
        z = state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & mask
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & mask
        out.append(z ^ (z >> 31))
    return out


def test_rotation_signs_are_bit63_of_the_published_stream():
    """Reading R9: sign -1 exactly when bit 63 of the output is set. The five published outputs
    at seed 1234567 give + + - + - (two of them are >= 2^63)."""
    vals = [int(l) for l in open(os.path.join(GOLDEN, "splitmix64_seed1234567.txt"))
            if l.strip() and not l.startswith("#")]
    want = [-1 if v >> 63 else 1 for v in vals]
    assert want == [1, 1, -1, 1, -1]
    S = O.rotation_signs(1234567, 1, 1, 5)
    assert S[0, 0, 0].tolist() == want


def test_rotation_signs_counter_layout_hand_computed():
    """Reading R9's counter ((t*l + f)*3 + r)*P + j, at L = 3, l = 2, P = 4, for elements whose
    counters are worked out by hand here: (t, f, r, j) = (1, 0, 2, 3) -> ((2 + 0)*3 + 2)*4 + 3
    = 35; (1, 1, 1, 2) -> ((2 + 1)*3 + 1)*4 + 2 = 42; (2, 1, 0, 1) -> ((4 + 1)*3 + 0)*4 + 1 = 61;
    (0, 1, 2, 0) -> ((0 + 1)*3 + 2)*4 + 0 = 20. The expected signs come from the stepped
    generator. The seed is chosen so that the plausible wrong layouts (r and j swapped in rank,
    table and function swapped, round outermost) give a different sign on at least one element."""
    seed = 20220601
    stream = _splitmix64_stepped(seed, 3 * 2 * 3 * 4)
    sign = [-1 if v >> 63 else 1 for v in stream]
    S = O.rotation_signs(seed, 3, 2, 4)
    cases = {(1, 0, 2, 3): 35, (1, 1, 1, 2): 42, (2, 1, 0, 1): 61, (0, 1, 2, 0): 20}
    for (t, f, r, j), c in cases.items():
        assert S[t, f, r, j] == sign[c], (t, f, r, j)
    # the same elements under wrong layouts read other counters with other signs
    wrong = [
        lambda t, f, r, j: ((t * 2 + f) * 4 + j) * 3 + r,       # j before r
        lambda t, f, r, j: ((f * 3 + t) * 3 + r) * 4 + j,       # function-major
        lambda t, f, r, j: ((r * 3 + t) * 2 + f) * 4 + j,       # round-major
    ]
    for w in wrong:
        assert any(sign[w(*e)] != sign[c] for e, c in cases.items())
    # and every element follows the stepped stream
    np.testing.assert_array_equal(S.reshape(-1), np.array(sign, dtype=np.int8))


def test_signs_balanced_and_seeded():
    S = O.rotation_signs(7, 4, 2, 256)
    assert S.shape == (4, 2, 3, 256)
    assert set(np.unique(S)) == {-1, 1}
    frac = np.mean(S == -1)
    assert abs(frac - 0.5) < 5 * 0.5 / math.sqrt(S.size)
    assert not np.array_equal(S, O.rotation_signs(8, 4, 2, 256))
    np.testing.assert_array_equal(S, O.rotation_signs(7, 4, 2, 256))


# ------------------------------------------------------------------ transform
@pytest.mark.parametrize("P", [2, 4, 8, 16, 64, 128, 512])
def test_fwht_equals_sylvester_matrix(P):
    rng = np.random.default_rng(P)
    V = rng.integers(-50, 51, size=(5, P)).astype(np.float32)   # exact in float32
    H = scipy.linalg.hadamard(P).astype(np.float64)
    np.testing.assert_array_equal(O.fwht_f32(V).astype(np.float64), V.astype(np.float64) @ H)


@pytest.mark.parametrize("P", [4, 64, 256, 4096])
def test_fwht_twice_is_P_identity(P):
    rng = np.random.default_rng(1)
    V = rng.integers(-8, 9, size=(3, P)).astype(np.float32)
    np.testing.assert_array_equal(O.fwht_f32(O.fwht_f32(V)), V * np.float32(P))


def test_fwht_preserves_norm_up_to_P():
    rng = np.random.default_rng(2)
    V = rng.standard_normal((20, 256)).astype(np.float32)
    W = O.fwht_f32(V).astype(np.float64)
    r = (W ** 2).sum(1) / (256.0 * (V.astype(np.float64) ** 2).sum(1))
    np.testing.assert_allclose(r, 1.0, rtol=1e-6)


def _rotation_matrix(signs_f, P):
    H = scipy.linalg.hadamard(P).astype(np.float64)
    R = np.eye(P)
    for r in range(3):
        R = H @ np.diag(signs_f[r].astype(np.float64)) @ R
    return R


@pytest.mark.parametrize("P", [8, 64, 256])
def test_rotation_is_scaled_orthogonal(P):
    S = O.rotation_signs(3, 1, 1, P)[0, 0]
    R = _rotation_matrix(S, P)
    np.testing.assert_array_equal(R.T @ R, (P ** 3) * np.eye(P))
    # the oracle's rotation applied to basis vectors reproduces the explicit product
    Y = O.rotate(np.eye(P, dtype=np.float32), S, P).astype(np.float64)
    np.testing.assert_array_equal(Y, R.T)   # row j of Y is R e_j


def test_rotation_matches_explicit_product_with_padding():
    d, D = 50, 64
    S = O.rotation_signs(11, 1, 1, 64)[0, 0]
    R = _rotation_matrix(S, 64)
    rng = np.random.default_rng(3)
    X = rng.standard_normal((10, d)).astype(np.float32)
    Xp = np.zeros((10, 64))
    Xp[:, :d] = X
    ref = Xp @ R.T
    got = O.rotate(X, S, D).astype(np.float64)
    assert np.max(np.abs(got - ref)) < 1e-5 * np.max(np.abs(ref))


# ------------------------------------------------------------------ code rule (Eq. 1)
def _preimage(S, P, v):
    """x with R x = v exactly: x = R^T v / P^3 (R has integer entries, P^3 a power of two)."""
    R = _rotation_matrix(S, P)
    x = (R.T @ v) / float(P ** 3)
    assert np.array_equal(x.astype(np.float32).astype(np.float64), x)
    return x.astype(np.float32)[None, :]


@pytest.mark.parametrize("P", [16, 64])
def test_code_of_basis_preimages(P):
    S = O.rotation_signs(5, 1, 1, P)
    for i in range(P):
        e = np.zeros(P)
        e[i] = 1.0
        assert O.hash_codes(_preimage(S[0, 0], P, e), S, P)[0, 0, 0] == i
        assert O.hash_codes(_preimage(S[0, 0], P, -e), S, P)[0, 0, 0] == i + P


def test_code_tie_rule_and_zero_vector():
    P = 16
    S = O.rotation_signs(9, 1, 1, P)
    code = lambda v: O.hash_codes(_preimage(S[0, 0], P, np.asarray(v, float)), S, P)[0, 0, 0]
    e = np.eye(P)
    assert code(e[3] + e[7]) == 3            # tie -> smaller index, positive -> +r
    assert code(-e[3] + e[7]) == 3 + P       # tie -> smaller index, negative -> -r
    assert code(e[3] - 2 * e[7]) == 7 + P
    assert O.hash_codes(np.zeros((1, P), np.float32), S, P)[0, 0, 0] == 0


# ------------------------------------------------------------------ index (Algorithm 1)
def _brute_top_pairs(X, signs_t, D, K):
    """All D^2 pairs scored from the raw projections with Python loops (reading R5)."""
    out = []
    y = [O.rotate(X, signs_t[f], D) for f in range(2)]
    for p in range(X.shape[0]):
        ranks = []
        for f in range(2):
            order = sorted(range(D), key=lambda i: (-abs(float(y[f][p, i])), i))
            ranks.append({i: r for r, i in enumerate(order)})
        cands = []
        for i in range(D):
            for j in range(D):
                s = np.float32(abs(y[0][p, i])) + np.float32(abs(y[1][p, j]))
                c1 = i if y[0][p, i] >= 0 else i + D
                c2 = j if y[1][p, j] >= 0 else j + D
                cands.append((-float(np.float32(s)), ranks[0][i], ranks[1][j], c1 * 2 * D + c2))
        cands.sort()
        out.append([c[3] for c in cands[:K]])
    return out


@pytest.mark.parametrize("K", [1, 2, 3, 5, 10])
def test_top_pairs_equal_full_enumeration(K):
    rng = np.random.default_rng(K)
    X = rng.standard_normal((60, 8)).astype(np.float32)
    D = 8
    S = O.rotation_signs(21, 1, 2, 8)[0]
    lists = [O.hash_lists(X, S[f], D) for f in range(2)]
    b, key = O.top_pairs(lists, D, K)
    assert b.tolist() == _brute_top_pairs(X, S, D, K)
    assert np.all(np.diff(key, axis=1) <= 0)


def test_top_pairs_with_exact_ties():
    # zero vectors: every pair scores 0, the position tie-break decides
    D = 8
    S = O.rotation_signs(1, 1, 2, 8)[0]
    X = np.zeros((2, 8), np.float32)
    lists = [O.hash_lists(X, S[f], D) for f in range(2)]
    b, _ = O.top_pairs(lists, D, 4)
    assert b.tolist() == _brute_top_pairs(X, S, D, 4)


def test_each_point_in_exactly_iprobes_distinct_buckets():
    rng = np.random.default_rng(4)
    X = rng.standard_normal((500, 32)).astype(np.float32)
    S = O.rotation_signs(2, 1, 2, 32)[0]
    lists = [O.hash_lists(X, S[f], 32) for f in range(2)]
    for K in (1, 3, 7):
        b, _ = O.top_pairs(lists, 32, K)
        assert b.shape == (500, K)
        assert all(len(set(row)) == K for row in b.tolist())
        assert b.min() >= 0 and b.max() < 64 * 64


def test_keep_count_values():
    k = lambda B, a, ip: int(O.keep_count(np.array([B]), a, ip)[0])
    assert k(10, 0.3, 3) == 1 and k(11, 0.3, 3) == 2 and k(0, 0.3, 3) == 0
    assert k(1, 0.5, 1) == 1 and k(2, 0.5, 1) == 1 and k(3, 0.5, 1) == 2
    assert k(7, 1.0, 1) == 7 and k(1, 0.01, 3) == 1
    assert int(O.keep_count(np.array([301]), 0.01, 1, "floor")[0]) == 3


def _uniform_data(n, d, seed):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((n, d))
    return (X / np.linalg.norm(X, axis=1, keepdims=True)).astype(np.float32)


@pytest.mark.parametrize("l", [1, 2])
def test_alpha1_iprobes1_is_a_partition_by_home_bucket(l):
    """Section 4: Falconn is Falconn++ with iProbes = 1 and alpha = 1."""
    X = _uniform_data(700, 24, 5)
    D = 16
    idx = O.build_index(X, L=3, D=D, alpha=1.0, iProbes=1, seed=13, l=l)
    codes = O.hash_codes(X, idx.signs, D)
    for t in range(3):
        ids = idx.ids[t]
        assert sorted(ids.tolist()) == list(range(700))
        home = codes[:, t, 0] if l == 1 else codes[:, t, 0] * (2 * D) + codes[:, t, 1]
        off = idx.offsets[t]
        for b in np.nonzero(np.diff(off))[0]:
            assert np.all(home[ids[off[b]:off[b + 1]]] == b)


@pytest.mark.parametrize("alpha,iprobes", [(0.3, 3), (0.5, 1), (0.1, 2)])
def test_filter_matches_per_bucket_brute_force(alpha, iprobes):
    X = _uniform_data(400, 16, 6)
    D = 8
    idx = O.build_index(X, L=2, D=D, alpha=alpha, iProbes=iprobes, seed=3, l=2)
    for t in range(2):
        lists = [O.hash_lists(X, idx.signs[t, f], D) for f in range(2)]
        b, key = O.top_pairs(lists, D, iprobes)
        buckets = {}
        for p in range(400):
            for r in range(iprobes):
                buckets.setdefault(int(b[p, r]), []).append((-float(key[p, r]), p))
        off, ids = idx.offsets[t], idx.ids[t]
        total = 0
        for bk in range(O.n_buckets(D, 2)):
            recs = sorted(buckets.get(bk, []))
            B = len(recs)
            keep = math.ceil(round(alpha * 1e6) * B / (iprobes * 1e6) - 1e-12) if B else 0
            assert off[bk + 1] - off[bk] == keep
            assert ids[off[bk]:off[bk + 1]].tolist() == [p for _, p in recs[:keep]]
            total += keep
        nonempty = len(buckets)
        assert alpha * 400 - 1e-9 <= total <= alpha * 400 + nonempty


# ------------------------------------------------------------------ heuristics and the LSF filter
def test_limit_scaling_keep_values():
    """max(kappa, keep(B)) records, never more than the bucket holds (Section 3.4, heuristic 2)."""
    got = O.keep_count(np.array([0, 1, 2, 5, 10, 100]), 0.3, 3, kappa=4)
    assert got.tolist() == [0, 1, 2, 4, 4, 10]
    assert O.keep_count(np.array([5, 100]), 0.3, 3, kappa=0).tolist() == [1, 10]


def test_limit_scaling_table_matches_per_bucket_brute_force():
    X = _uniform_data(400, 16, 61)
    D, K, alpha, kappa = 8, 2, 0.1, 3
    idx = O.build_index(X, L=1, D=D, alpha=alpha, iProbes=K, seed=5, l=2, kappa=kappa)
    lists = [O.hash_lists(X, idx.signs[0, f], D) for f in range(2)]
    b, key = O.top_pairs(lists, D, K)
    buckets = {}
    for p in range(400):
        for r in range(K):
            buckets.setdefault(int(b[p, r]), []).append((-float(key[p, r]), p))
    off, ids = idx.offsets[0], idx.ids[0]
    for bk in range(O.n_buckets(D, 2)):
        recs = sorted(buckets.get(bk, []))
        B = len(recs)
        keep = min(B, max(kappa, math.ceil(round(alpha * 1e6) * B / (K * 1e6) - 1e-12))) if B else 0
        assert off[bk + 1] - off[bk] == keep
        assert ids[off[bk]:off[bk + 1]].tolist() == [p for _, p in recs[:keep]]


def test_center_vector_is_the_mean():
    rng = np.random.default_rng(62)
    X = rng.standard_normal((3000, 7)).astype(np.float32) + np.float32(0.25)
    c = O.center_vector(X, chunk=1000)
    for j in range(7):
        exact = math.fsum(float(v) for v in X[:, j]) / 3000
        assert abs(float(c[j]) - exact) <= 1.5 * np.spacing(np.float32(abs(exact)))
    # the running sum in row order, whatever the chunking
    assert np.array_equal(c, O.center_vector(X, chunk=7))


def test_centering_symmetric_data_changes_nothing():
    """X together with -X has centre 0 exactly, so the centred index is the plain one."""
    X = _uniform_data(150, 16, 63)
    X2 = np.concatenate([X, -X])
    assert not O.center_vector(X2).any()
    a = O.build_index(X2, L=2, D=8, alpha=0.5, iProbes=2, seed=4, l=2, center=True)
    b = O.build_index(X2, L=2, D=8, alpha=0.5, iProbes=2, seed=4, l=2)
    for t in range(2):
        assert np.array_equal(a.offsets[t], b.offsets[t]) and np.array_equal(a.ids[t], b.ids[t])


def test_centering_hashes_x_minus_c_and_keeps_the_argmax():
    rng = np.random.default_rng(64)
    X = rng.standard_normal((500, 16))
    X = (X / np.linalg.norm(X, axis=1, keepdims=True) + 0.5).astype(np.float32)
    idx = O.build_index(X, L=1, D=8, alpha=1.0, iProbes=1, seed=6, l=1, center=True)
    c = O.center_vector(X)
    Xc = (X - c).astype(np.float32)
    home = O.hash_codes(Xc, idx.signs, 8)[:, 0, 0]
    off = idx.offsets[0]
    for bk in np.nonzero(np.diff(off))[0]:
        assert np.all(home[idx.ids[0][off[bk]:off[bk + 1]]] == bk)
    # argmax x^T q = argmax (x - c)^T q (Section 3.4): the same top-5 by exact scores
    q = rng.standard_normal(16)
    X64, c64 = X.astype(np.float64), c.astype(np.float64)
    assert np.array_equal(np.argsort(-(X64 @ q))[:5], np.argsort(-((X64 - c64) @ q))[:5])


@pytest.mark.parametrize("l", [1, 2])
def test_lsf_threshold_tail_probability(l):
    """Pr[N(0,1) >= t]^l = alpha / (2D)^l (checked with math.erfc), on the |y| scale P."""
    alpha, D, P = 0.1, 16, 32
    T = O.lsf_threshold(alpha, D, l, P)
    t = float(T) / P
    tail = 0.5 * math.erfc(t / math.sqrt(2.0))
    assert abs(tail ** l - float(np.float32(alpha)) / (2 * D) ** l) <= 1e-6 * float(np.float32(alpha)) / (2 * D) ** l


def test_threshold_filter_keeps_records_above_the_bound():
    X = _uniform_data(300, 16, 65)
    D, K = 8, 3
    idx = O.build_index(X, L=1, D=D, alpha=0.2, iProbes=K, seed=7, l=2, filter="threshold", threshold=0.8)
    T = np.float32(16 * float(np.float32(0.8)))
    assert idx.threshold == T
    lists = [O.hash_lists(X, idx.signs[0, f], D) for f in range(2)]
    b, key = O.top_pairs(lists, D, K)
    want = {}
    for p in range(300):
        for r in range(K):
            # positions of the pair in the two lists: recover |y1|, |y2| by code
            c1, c2 = divmod(int(b[p, r]), 2 * D)
            a1 = lists[0].a[p][list(lists[0].code[p]).index(c1)]
            a2 = lists[1].a[p][list(lists[1].code[p]).index(c2)]
            if a1 >= T and a2 >= T:
                want.setdefault(int(b[p, r]), []).append((-float(key[p, r]), p))
    off, ids = idx.offsets[0], idx.ids[0]
    for bk in range(O.n_buckets(D, 2)):
        recs = sorted(want.get(bk, []))
        assert ids[off[bk]:off[bk + 1]].tolist() == [p for _, p in recs]


def test_threshold_zero_keeps_every_record():
    """A bound below every projection keeps all records: with iProbes = 1 that is the alpha = 1
    table (plain cross-polytope LSH)."""
    X = _uniform_data(300, 16, 66)
    a = O.build_index(X, L=2, D=8, alpha=0.3, iProbes=1, seed=8, l=2, filter="threshold", threshold=1e-30)
    b = O.build_index(X, L=2, D=8, alpha=1.0, iProbes=1, seed=8, l=2)
    for t in range(2):
        assert np.array_equal(a.offsets[t], b.offsets[t]) and np.array_equal(a.ids[t], b.ids[t])


# ------------------------------------------------------------------ SimHash store
def test_simhash_bits_agree_with_the_hash_codes():
    """The sign bit of a function's top index is set exactly when its code is i + D (Eq. 1)."""
    X = _uniform_data(300, 32, 70)
    S = O.rotation_signs(3, 2, 2, 32)
    bits = O.simhash_bits(X, S, 32, 4)
    for g in range(4):
        t, f = divmod(g, 2)
        h = O.hash_lists(X, S[t, f], 32)
        top = h.idx[:, 0]
        assert np.array_equal(bits[np.arange(300), g * 32 + top], h.code[:, 0] >= 32)


def test_simhash_hamming_estimates_the_angle():
    """For random rotations the fraction of differing signs estimates angle / pi (SimHash)."""
    rng = np.random.default_rng(71)
    d, F, D = 64, 16, 64
    S = O.rotation_signs(9, F, 1, d)
    for cos in (0.9, 0.5, 0.0):
        fr = []
        for _ in range(40):
            a = rng.standard_normal(d)
            a /= np.linalg.norm(a)
            z = rng.standard_normal(d)
            z -= (z @ a) * a
            z /= np.linalg.norm(z)
            b = cos * a + math.sqrt(1 - cos * cos) * z
            bits = O.simhash_bits(np.stack([a, b]), S, D, F)
            fr.append(np.mean(bits[0] != bits[1]))
        assert abs(np.mean(fr) - math.acos(cos) / math.pi) < 0.04, (cos, np.mean(fr))


def test_simhash_score_extremes_and_packing():
    X = _uniform_data(20, 16, 72)
    S = O.rotation_signs(4, 2, 2, 16)
    bits = O.simhash_bits(X, S, 16, 4)
    neg = O.simhash_bits(-X, S, 16, 4)
    assert np.all(O.simhash_score(bits, bits[0])[0] == 64)
    assert O.simhash_score(neg[:1], bits[0])[0] == -64          # every sign flips
    w = O.simhash_words(bits)
    for r in range(3):
        for b in range(64):
            assert ((int(w[r, b // 32]) >> (b % 32)) & 1) == int(bits[r, b])


def test_simhash_rerank_with_full_short_list_equals_plain_query():
    X = _uniform_data(400, 16, 73)
    idx = O.build_index(X, L=3, D=8, alpha=0.5, iProbes=2, seed=12, l=2)
    Q = _uniform_data(5, 16, 74)
    ids, sc, _ = O.query_reranked(idx, Q, 5, 40, R=400, storage="simhash", simhash_functions=4)
    pid, psc, _ = O.query(idx, Q, 5, 40)
    assert np.array_equal(ids, pid)


# ------------------------------------------------------------------ query
def _brute_probes(idx, q, qProbes, gap=False):
    D, L = idx.D, idx.L
    cands = []
    for t in range(L):
        y = [O.rotate(q[None, :], idx.signs[t, f], D)[0] for f in range(2)]
        ranks = []
        for f in range(2):
            order = sorted(range(D), key=lambda i: (-abs(float(y[f][i])), i))
            ranks.append({i: r for r, i in enumerate(order)})
        best = max(np.float32(np.float32(abs(y[0][i])) + np.float32(abs(y[1][j])))
                   for i in range(D) for j in range(D))
        for i in range(D):
            for j in range(D):
                s = np.float32(np.float32(abs(y[0][i])) + np.float32(abs(y[1][j])))
                if gap:      # plain Falconn: the loss against the table's best pair
                    s = np.float32(s - best)
                s = float(s)
                c1 = i if y[0][i] >= 0 else i + D
                c2 = j if y[1][j] >= 0 else j + D
                cands.append((-s, t, ranks[0][i], ranks[1][j], t * 4 * D * D + c1 * 2 * D + c2))
    cands.sort()
    return [c[4] for c in cands[:qProbes]]


@pytest.mark.parametrize("qProbes", [1, 5, 37, 10_000])
def test_probe_ranking_equals_enumeration(qProbes):
    X = _uniform_data(50, 12, 7)
    idx = O.build_index(X, L=3, D=4, alpha=0.5, iProbes=2, seed=5, l=2)
    q = _uniform_data(1, 12, 8)[0]
    assert O.probes(idx, q, qProbes).tolist() == _brute_probes(idx, q, qProbes)


@pytest.mark.parametrize("qProbes", [1, 3, 5, 37, 10_000])
def test_gap_probe_ranking_equals_enumeration(qProbes):
    X = _uniform_data(50, 12, 7)
    idx = O.build_index(X, L=3, D=4, alpha=0.5, iProbes=2, seed=5, l=2)
    q = _uniform_data(1, 12, 9)[0]
    assert O.probes(idx, q, qProbes, "gap").tolist() == _brute_probes(idx, q, qProbes, gap=True)


def test_gap_probing_takes_each_tables_best_bucket_first():
    """With qProbes <= L the gap score (0 for every table's best pair) selects the home bucket of
    the first qProbes tables, as plain Falconn does before any second probe."""
    X = _uniform_data(200, 16, 10)
    idx = O.build_index(X, L=6, D=8, alpha=1.0, iProbes=1, seed=11, l=2)
    q = _uniform_data(1, 16, 12)[0]
    home = O.hash_codes(q[None, :], idx.signs, 8)[0]
    NB = O.n_buckets(8, 2)
    for qp in (1, 4, 6):
        got = O.probes(idx, q, qp, "gap").tolist()
        assert got == [t * NB + int(home[t, 0]) * 16 + int(home[t, 1]) for t in range(qp)]


def test_full_probing_reaches_every_sign_consistent_point():
    """Probing all L * D^l pairs visits, per table, every bucket whose wedges lie on the query's
    side of each random vector (Eq. 1 picks +r_i or -r_i by the sign of the projection). With
    alpha = 1 and iProbes = 1 the candidates are exactly the points whose home bucket is such a
    bucket in some table, and the answer is brute force over those points."""
    X = _uniform_data(300, 20, 9)
    Q = _uniform_data(15, 20, 10)
    for l, D in ((1, 16), (2, 8)):
        idx = O.build_index(X, L=2, D=D, alpha=1.0, iProbes=1, seed=1, l=l)
        ids, sc, st = O.query(idx, Q, 10, qProbes=10 ** 9)
        codes = O.hash_codes(X, idx.signs, D)
        for r in range(Q.shape[0]):
            members = []
            for p in range(300):
                hit = False
                for t in range(2):
                    ok = True
                    for f in range(l):
                        yq = O.rotate(Q[r:r + 1], idx.signs[t, f], D)[0]
                        c = int(codes[p, t, f])
                        ok = ok and ((c < D) == bool(yq[c % D] >= 0))
                    hit = hit or ok
                if hit:
                    members.append(p)
            assert st[r, 2] == len(members)
            members = np.array(members, dtype=np.int64)
            bi, bs = O.brute_force(X[members], Q[r:r + 1], 10)
            ref = np.where(bi[0] >= 0, members[np.maximum(bi[0], 0)], -1)
            assert ids[r].tolist() == ref.tolist()
            np.testing.assert_array_equal(sc[r], bs[0])


def test_brute_force_equals_enumeration():
    X = _uniform_data(1500, 10, 11)
    X[7] = X[3]          # a duplicate point: the id tie-break must apply
    Q = _uniform_data(6, 10, 12)
    Q[0] = X[3]
    bi, bs = O.brute_force(X, Q, 12)
    for r in range(6):
        sc = [(-math.fsum(float(a) * float(b) for a, b in zip(X[i], Q[r])), i) for i in range(1500)]
        sc.sort()
        assert bi[r].tolist() == [i for _, i in sc[:12]]
        np.testing.assert_allclose(bs[r], [-s for s, _ in sc[:12]], rtol=0, atol=1e-15)
    assert bi[0, 0] == 3 and bi[0, 1] == 7


def test_short_results_are_padded():
    X = _uniform_data(5, 8, 13)
    idx = O.build_index(X, L=1, D=8, alpha=1.0, iProbes=1, seed=2, l=1)
    ids, sc, _ = O.query(idx, X[:1], 10, qProbes=1)
    n_found = int((ids[0] >= 0).sum())
    assert n_found >= 1 and np.all(ids[0, n_found:] == -1) and np.all(np.isneginf(sc[0, n_found:]))
    assert ids[0, 0] == 0


def test_recall():
    t = np.array([[1, 2, 3, 4]])
    assert O.recall_at_k(np.array([[4, 3, 9, -1]]), t) == 0.5
    assert O.recall_at_k(t, t) == 1.0


def test_lemma2_projection_on_argmax_vector_statistical():
    """Loose sanity of Lemma 2 (CEOs): with r_i scaled to Gaussian length (rows of R have norm
    P^{3/2}, a Gaussian vector about sqrt(P), so y / P), x^T r_1 has mean near rho * sqrt(2 ln D)."""
    P = D = 1024
    rng = np.random.default_rng(14)
    S = O.rotation_signs(4, 200, 1, P)
    rho = 0.8
    vals = []
    for t in range(200):
        q = rng.standard_normal(P)
        q /= np.linalg.norm(q)
        z = rng.standard_normal(P)
        z -= (z @ q) * q
        z /= np.linalg.norm(z)
        x = rho * q + math.sqrt(1 - rho ** 2) * z
        yq = O.rotate(q[None].astype(np.float32), S[t, 0], D)[0].astype(np.float64)
        yx = O.rotate(x[None].astype(np.float32), S[t, 0], D)[0].astype(np.float64)
        i = int(np.argmax(np.abs(yq)))
        vals.append(np.sign(yq[i]) * yx[i] / P)
    mean = float(np.mean(vals))
    # Lemma 2 is asymptotic in D; at D = 1024 the extreme-value mean sits below sqrt(2 ln D)
    assert 0.75 * rho * math.sqrt(2 * math.log(D)) < mean < 1.05 * rho * math.sqrt(2 * math.log(D))


# ------------------------------------------------------------------ quantisers
def test_bf16_matches_torch_rne():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(15)
    x = rng.standard_normal(20000).astype(np.float32)
    # exact halfway cases: low 16 bits = 0x8000 with both parities of bit 16
    u = rng.integers(0, 2 ** 31, 2000, dtype=np.uint64).astype(np.uint32)
    u = (u & np.uint32(0x7F7F0000)) | np.uint32(0x8000)
    x = np.concatenate([x, u.view(np.float32), -u.view(np.float32), [0.0, -0.0]]).astype(np.float32)
    ref = torch.from_numpy(x).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    np.testing.assert_array_equal(O.bf16_bits(x), ref)


def test_e4m3_matches_torch_and_table():
    torch = pytest.importorskip("torch")
    if not hasattr(torch, "float8_e4m3fn"):
        pytest.skip("torch without float8_e4m3fn")
    rng = np.random.default_rng(16)
    vals = O.e4m3_value(np.arange(127, dtype=np.uint8)).astype(np.float64)
    mids = (vals[:-1] + vals[1:]) / 2
    x = np.concatenate([rng.uniform(-448, 448, 20000), vals, -vals, mids, -mids,
                        rng.uniform(-0.02, 0.02, 5000)]).astype(np.float32)
    ref = torch.from_numpy(x).to(torch.float8_e4m3fn).view(torch.uint8).numpy()
    np.testing.assert_array_equal(O.e4m3_bits(x), ref)
    # decode: torch's widening cast of every finite code
    codes = np.array([c for c in range(256) if (c & 0x7F) != 0x7F], dtype=np.uint8)
    dec = torch.from_numpy(codes).view(torch.float8_e4m3fn).to(torch.float32).numpy()
    np.testing.assert_array_equal(O.e4m3_value(codes), dec)
    assert O.e4m3_value(np.array([0x7E], np.uint8))[0] == 448.0
    assert O.e4m3_bits(np.array([1000.0, -1e6], np.float32)).tolist() == [0x7E, 0xFE]


def test_fp8_rows_scale_and_zero_vector():
    X = _uniform_data(50, 33, 17)
    X[4] = 0.0
    codes, s = O.quantize_fp8_rows(X)
    assert s[4] == 1.0 and np.all(codes[4] == 0)
    mx = np.max(np.abs(O.e4m3_value(codes)), axis=1)
    assert np.all(mx[np.arange(50) != 4] == 448.0)
    deq = O.dequantized_store(X, "fp8")
    rel = np.abs(deq - X) / np.max(np.abs(X), axis=1, keepdims=True).clip(1e-30)
    assert rel[np.arange(50) != 4].max() <= 2.0 ** -4 * 1.0001   # half an ulp at the top binade


@pytest.mark.parametrize("storage", ["bf16", "fp8"])
def test_rerank_with_full_short_list_equals_plain_query(storage):
    X = _uniform_data(400, 16, 18)
    Q = _uniform_data(8, 16, 19)
    idx = O.build_index(X, L=4, D=8, alpha=0.5, iProbes=2, seed=4, l=2)
    pi, ps, st = O.query(idx, Q, 10, qProbes=30)
    ri, rs, short = O.query_reranked(idx, Q, 10, qProbes=30, R=400, storage=storage)
    np.testing.assert_array_equal(pi, ri)
    np.testing.assert_array_equal(ps, rs)


def test_chunked_hashing_gives_the_same_table():
    """build_table hashes rows in chunks; every row's hash depends on that row alone, so a chunk of
    7 rows and one chunk of all rows give identical tables."""
    X = _uniform_data(300, 20, 81)
    S = O.rotation_signs(3, 1, 2, 32)
    a = O.build_table(X, S[0], 16, 2, 0.4, 3)
    b = O.build_table(X, S[0], 16, 2, 0.4, 3, chunk=7)
    for u, v in zip(a, b):
        np.testing.assert_array_equal(u, v)


@pytest.mark.parametrize("storage", ["bf16", "fp8"])
def test_rerank_short_list_cut_by_approximate_score(storage):
    """With R < |C| the short list is the first R candidates by (approximate score desc, id asc)
    and the answer is the exact top-k of that list. Checked against a Python enumeration that
    takes the dequantised values from torch's own casts (a library routine) and sums products
    with math.fsum; the data makes the approximate and the exact top-R differ, so ordering the
    short list by the exact score, or ascending, fails."""
    torch = pytest.importorskip("torch")
    # tight clusters: neighbours' scores differ by less than the quantisation error
    rng = np.random.default_rng(91)
    base = _uniform_data(4, 24, 92).astype(np.float64)
    X = base[rng.integers(0, 4, size=600)] + 0.004 * rng.standard_normal((600, 24))
    X = (X / np.linalg.norm(X, axis=1, keepdims=True)).astype(np.float32)
    Q = base[np.arange(12) % 4] + 0.004 * rng.standard_normal((12, 24))
    Q = (Q / np.linalg.norm(Q, axis=1, keepdims=True)).astype(np.float32)
    idx = O.build_index(X, L=4, D=8, alpha=0.6, iProbes=2, seed=5, l=2)
    R, k = 6, 3
    ids, sc, short = O.query_reranked(idx, Q, k, qProbes=40, R=R, storage=storage)
    if storage == "bf16":
        deq = torch.from_numpy(X).to(torch.bfloat16).to(torch.float64).numpy()
    else:
        s = (np.max(np.abs(X), axis=1) / np.float32(448.0)).astype(np.float32)
        codes = torch.from_numpy((X / s[:, None]).astype(np.float32)).to(torch.float8_e4m3fn)
        deq = codes.to(torch.float64).numpy() * s.astype(np.float64)[:, None]
    differs = 0
    for r in range(Q.shape[0]):
        cand = O.candidates(idx, O.probes(idx, Q[r], 40))
        assert len(cand) > R
        q = [float(v) for v in Q[r]]
        approx = {int(c): math.fsum(float(deq[c, j]) * q[j] for j in range(24)) for c in cand}
        exact = {int(c): math.fsum(float(X[c, j]) * q[j] for j in range(24)) for c in cand}
        want = sorted(approx, key=lambda c: (-approx[c], c))[:R]
        assert short[r].tolist() == want, r
        top = sorted(want, key=lambda c: (-exact[c], c))[:k]
        assert ids[r].tolist() == top
        np.testing.assert_allclose(sc[r], [exact[c] for c in top], rtol=1e-15, atol=1e-15)
        differs += set(want) != set(sorted(exact, key=lambda c: (-exact[c], c))[:R])
    assert differs > 0
