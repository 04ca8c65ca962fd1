"""Plain CPU oracle of the Falconn++ hot path. TEST INFRASTRUCTURE ONLY.

Only the test-suite, the package smoke check and the benchmark's CPU-baseline
leg may import this module. The product path (the HIP library and its Python
binding) never calls it, and this module never imports the product path.

What it computes (Pham & Liu, "Falconn++", NeurIPS 2022):

* the cross-polytope hash of Section 2.2 (Eq. 1), evaluated with the
  structured-spinner rotation the paper names in Section 3.4: three rounds of a
  random +-1 diagonal followed by an unnormalised fast Walsh-Hadamard transform;
* l concatenated hashes per table (Section 4, "parameter settings": l = 2,
  4D^2 buckets);
* multi-probe indexing and the per-bucket alpha-fraction filter (Algorithm 1,
  Section 3.4 "practical implementation");
* multi-probe querying ranked by |q^T r_i| over all L tables (Section 3.4,
  "multi-probing for querying"; Section 2.2 for qProbes being a total);
* candidate union, inner-product scoring and top-k (problem statement in
  Section 1);
* brute force and recall (Section 4);
* the BF16 / FP8-E4M3 scoring stores with an exact rerank of a short list
  (an addition on top of the paper; the quantisers are the standard
  round-to-nearest-even definitions).

Hashing is evaluated in float32 with a fixed butterfly order (stage h = 1, 2,
4, ..., P/2; pair (j, j+h) -> (v_j + v_{j+h}, v_j - v_{j+h})), so its codes are
bit-comparable with any other implementation that keeps that expression tree.
Scores are float64.

Readings where the paper is silent (every one is also listed in the design notes):

R1  P = max(D, 2^ceil(log2 d)); x is zero-padded to P; the first D outputs are the projections.
R2  No normalisation of the transform (the argmax and all rankings are scale-invariant).
R3  Argmax ties go to the smallest index; y_i >= 0 (so -0.0 too) gives code i, else i + D (Eq. 1).
R4  Per function, the list Lambda orders the D indices by (|y_i| desc, i asc).
R5  l = 2: bucket = c1 * 2D + c2; the pair score is the float32 sum |y1| + |y2|; pairs are
    ranked by (score desc, position in Lambda1 asc, position in Lambda2 asc).
R6  keep(B) = ceil(A*B / (iProbes * 10^6)) with A = floor(alpha * 10^6 + 1/2), exact integers;
    kept records are ordered by (key desc, id asc).
R7  qProbes is the total over all tables; probes are ranked by (score desc, table asc, pos1 asc, pos2 asc).
R8  Top-k order is (score desc, id asc); short results are padded with (-1, -inf).
R9  Signs: S_{t,f,r}[j] = -1 iff bit 63 of SplitMix64 at counter ((t*l + f)*3 + r)*P + j is set.
R15 Centering: c_j = fl32(running float64 sum of x_ij over rows in order / n); the build hashes
    fl32(x - c); queries are hashed unchanged; scores are x^T q on the uncentred data.
R16 Global threshold: keep a record when each |y| of its pair is >= fl32(P * t) with
    t = Phi^-1(1 - alpha^(1/l) / (2D)) (sqrt for l = 2), or a given t.
R18 SimHash store: bit g*D + i of a signature is the sign (y_i < 0) of projection i of hash
    function g = t*l + f, for the first F functions; approximate score = F*D - 2 * Hamming;
    data signatures use the uncentred vectors (the queries' rotation).
R17 Gap probing (plain Falconn): a pair's probe score is fl32(s - s_top) with s its pair score
    and s_top = fl32(a_0 + b_0) its table's best (l = 1: fl32(a_i - a_0)), so the cost of a bucket
    is the loss of projection summed over the functions; ranked as R7.

Parity pinned: every function below is pinned by a test against a closed form,
an invariant stated by the paper, a special case, or brute-force enumeration.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# ----------------------------------------------------------------------------------------------
# Random signs: SplitMix64 (S. Vigna's published generator), used as a counter-based stream.
# ----------------------------------------------------------------------------------------------
_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64_at(seed: int, counter: np.ndarray) -> np.ndarray:
    """Output number ``counter`` (0-based) of a SplitMix64 stream started at state ``seed``.

    SplitMix64 advances its state by the golden-ratio constant and then mixes:
    z = (z ^ (z >> 30)) * M1; z = (z ^ (z >> 27)) * M2; out = z ^ (z >> 31).
    Output c therefore mixes the state seed + (c + 1) * golden (mod 2^64).
    """
    c = np.asarray(counter, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + (c + np.uint64(1)) * _GOLDEN
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def rotation_signs(seed: int, L: int, l: int, P: int) -> np.ndarray:
    """Random diagonals of the structured spinner: int8 array [L][l][3][P] of +-1 (reading R9)."""
    c = np.arange(L * l * 3 * P, dtype=np.uint64)
    z = splitmix64_at(seed, c)
    s = np.where((z >> np.uint64(63)) != 0, -1, 1).astype(np.int8)
    return s.reshape(L, l, 3, P)


# ----------------------------------------------------------------------------------------------
# Rotation (Section 3.4: structured spinners built from the fast Hadamard transform).
# ----------------------------------------------------------------------------------------------
def padded_dim(d: int, D: int) -> int:
    """Reading R1: the transform length P = max(D, next power of two >= d)."""
    p = 1
    while p < d:
        p *= 2
    return max(p, D)


def fwht_f32(V: np.ndarray) -> np.ndarray:
    """Unnormalised Sylvester-order Walsh-Hadamard transform of each row, in float32.

    Stage h = 1, 2, 4, ..., P/2: every j with (j & h) == 0 becomes v_j + v_{j+h}
    and j + h becomes v_j - v_{j+h}; each operation rounds to float32.
    """
    V = np.array(V, dtype=np.float32, copy=True)
    m, P = V.shape
    h = 1
    while h < P:
        W = V.reshape(m, P // (2 * h), 2, h)
        a = W[:, :, 0, :].copy()
        b = W[:, :, 1, :].copy()
        W[:, :, 0, :] = a + b
        W[:, :, 1, :] = a - b
        h *= 2
    return V


def rotate(X: np.ndarray, signs_f: np.ndarray, D: int) -> np.ndarray:
    """Projections y = (H S3 H S2 H S1 pad(x))[0:D] for each row, in float32 (rounds r = 0, 1, 2)."""
    n, d = X.shape
    P = signs_f.shape[-1]
    V = np.zeros((n, P), dtype=np.float32)
    V[:, :d] = X
    for r in range(3):
        V = V * signs_f[r].astype(np.float32)   # exact: multiplication by +-1
        V = fwht_f32(V)
    return V[:, :D]


@dataclass
class HashLists:
    """Per-vector sorted projection lists of one hash function (reading R4).

    idx[v, p]  : the index i of the p-th largest |y_i| (ties by smaller i)
    a[v, p]    : |y_idx| (float32)
    code[v, p] : idx if y_idx >= 0 else idx + D   (Eq. 1 with reading R3)
    """

    idx: np.ndarray
    a: np.ndarray
    code: np.ndarray


def hash_lists(X: np.ndarray, signs_f: np.ndarray, D: int) -> HashLists:
    y = rotate(X, signs_f, D)
    a = np.abs(y)
    i = np.arange(D, dtype=np.int64)
    code_all = np.where(y >= np.float32(0.0), i[None, :], i[None, :] + D)
    order = np.argsort(-a, axis=1, kind="stable")     # |y| desc, ties keep i ascending
    return HashLists(idx=order,
                     a=np.take_along_axis(a, order, axis=1),
                     code=np.take_along_axis(code_all, order, axis=1))


def hash_codes(X: np.ndarray, signs: np.ndarray, D: int) -> np.ndarray:
    """Cross-polytope code of every vector under every function: int32 [n][L][l] (Eq. 1)."""
    L, l = signs.shape[:2]
    out = np.empty((X.shape[0], L, l), dtype=np.int32)
    for t in range(L):
        for f in range(l):
            out[:, t, f] = hash_lists(X, signs[t, f], D).code[:, 0]
    return out


# ----------------------------------------------------------------------------------------------
# Index (Algorithm 1 with l concatenated functions).
# ----------------------------------------------------------------------------------------------
def n_buckets(D: int, l: int) -> int:
    return (2 * D) ** l


def top_pairs(lists, D: int, K: int, with_parts: bool = False):
    """Top-K buckets of every vector under one table (Algorithm 1, first loop; reading R5).

    Returns bucket [n][K] int64 and key [n][K] float32, best first.
    For l = 1 the candidates are the list entries themselves (score |y_i|).
    For l = 2 a pair at list positions (i, j) has score fl32(a1_i + a2_j). Every pair
    with i >= K or j >= K is preceded by at least K pairs of the same column or row
    (the score cannot increase along a sorted list, and the position tie-break favours
    the smaller position), so only positions below min(K, D) need to be enumerated.
    """
    if len(lists) == 1:
        h = lists[0]
        out = (h.code[:, :K].astype(np.int64), h.a[:, :K].copy())
        return out + ((h.a[:, :K].copy(),),) if with_parts else out
    h1, h2 = lists
    Kc = min(K, D)
    n = h1.a.shape[0]
    s = (h1.a[:, :Kc, None] + h2.a[:, None, :Kc]).astype(np.float32)      # [n][Kc][Kc]
    b = h1.code[:, :Kc, None].astype(np.int64) * (2 * D) + h2.code[:, None, :Kc]
    s = s.reshape(n, Kc * Kc)
    b = b.reshape(n, Kc * Kc)
    # order by (score desc, flat position asc); flat position = i*Kc + j is (i, j) lexicographic
    order = np.argsort(-s, axis=1, kind="stable")[:, :K]
    out = (np.take_along_axis(b, order, axis=1), np.take_along_axis(s, order, axis=1))
    if not with_parts:
        return out
    a1 = np.repeat(h1.a[:, :Kc], Kc, axis=1)            # flat (i, j) -> a1[i]
    a2 = np.tile(h2.a[:, :Kc], (1, Kc))                 # flat (i, j) -> a2[j]
    return out + ((np.take_along_axis(a1, order, axis=1), np.take_along_axis(a2, order, axis=1)),)


def alpha_micro(alpha: float) -> int:
    """alpha as an integer number of millionths: A = floor(alpha * 10^6 + 1/2) (reading R6)."""
    return int(math.floor(float(np.float32(alpha)) * 1e6 + 0.5))


def keep_count(B: np.ndarray, alpha: float, iProbes: int, rounding: str = "ceil",
               kappa: int = 0) -> np.ndarray:
    """Reading R6 of 'keep the top-(alpha B / iProbes) points' (Algorithm 1, last line).

    keep(B) = ceil(A * B / (iProbes * 10^6)) in exact integers, A = alpha in millionths,
    so a decimal alpha such as 0.3 behaves as written (0.3 * 10 / 3 keeps exactly 1).
    Limit scaling (Section 3.4, heuristic 2) keeps max(kappa, keep(B)) records, and never more
    than the bucket holds: min(B, max(kappa, keep(B))).
    """
    A = alpha_micro(alpha)
    den = int(iProbes) * 1_000_000
    B = np.asarray(B, dtype=np.int64)
    num = B * A
    if rounding == "ceil":
        out = (num + (den - 1)) // den
    else:
        out = num // den
    if kappa > 0:
        out = np.maximum(out, np.minimum(B, kappa))
    return out.astype(np.int64)


def center_vector(X: np.ndarray, chunk: int = 1 << 16) -> np.ndarray:
    """Centre of the data (Section 3.4, heuristic 1): c = sum_i x_i / n (reading R15).

    Per coordinate the float64 sum runs over the rows in order (a running sum), is divided by
    n in float64 and rounded to float32.
    """
    X = np.asarray(X, dtype=np.float32)
    run = np.zeros((1, X.shape[1]), dtype=np.float64)
    for r0 in range(0, X.shape[0], chunk):
        run = np.cumsum(np.vstack([run, X[r0:r0 + chunk].astype(np.float64)]), axis=0)[-1:]
    return (run[0] / float(X.shape[0])).astype(np.float32)


def lsf_threshold(alpha: float, D: int, l: int, P: int) -> np.float32:
    """Global threshold of the theoretical LSF filter (appendix, Falconn++ vs. theoretical LSF):
    t with Pr[N(0,1) >= t]^l = alpha / (2D)^l, i.e. t = Phi^-1(1 - alpha^(1/l) / (2D)), on the
    scale of the unnormalised rotation (a unit vector's projections have standard deviation P):
    the float32 bound P * t on |y| (reading R16)."""
    from scipy.stats import norm
    a = float(np.float32(alpha))
    p = (a if l == 1 else float(np.sqrt(a))) / (2.0 * D)
    t = float(norm.isf(p))
    return np.float32(max(0.0, float(P) * t))


@dataclass
class Index:
    X: np.ndarray
    L: int
    D: int
    l: int
    P: int
    alpha: float
    iProbes: int
    seed: int
    signs: np.ndarray
    offsets: list = field(default_factory=list)    # per table: int64 [NB + 1]
    ids: list = field(default_factory=list)        # per table: int32 [table size]
    keys: list = field(default_factory=list)       # per table: float32 [table size] (the kept keys)
    center: np.ndarray | None = None               # centring vector of a centred build
    threshold: np.float32 | None = None            # bound on |y| of a threshold-filter build


def build_table(X, signs_t, D, l, alpha, iProbes, rounding="ceil", kappa=0, threshold=None,
                chunk=1 << 17):
    """One hash table: hash, top-iProbes buckets per point, per-bucket filter, CSR.

    threshold (float32 bound on |y|): the global-threshold filter keeps a record when each of
    its l projections is >= the bound, and every bucket keeps all such records.
    Points are hashed `chunk` rows at a time (each row's hash depends on that row alone), which
    bounds the memory of the sorted lists.
    """
    n = X.shape[0]
    pieces = []
    for r0 in range(0, n, chunk):
        lists = [hash_lists(X[r0:r0 + chunk], signs_t[f], D) for f in range(l)]
        pieces.append(top_pairs(lists, D, iProbes, with_parts=threshold is not None))
    bucket = np.concatenate([p[0] for p in pieces])
    key = np.concatenate([p[1] for p in pieces])
    if threshold is not None:
        parts = tuple(np.concatenate([p[2][f] for p in pieces]) for f in range(l))
    K = bucket.shape[1]
    rb = bucket.reshape(-1)
    rk = key.reshape(-1)
    rid = np.repeat(np.arange(n, dtype=np.int64), K)
    if threshold is not None:
        ok = np.ones(rb.shape[0], dtype=bool)
        for part in parts:
            ok &= part.reshape(-1) >= np.float32(threshold)
        rb, rk, rid = rb[ok], rk[ok], rid[ok]
    # records ordered by (bucket asc, key desc, id asc)
    order = np.lexsort((rid, -rk, rb))
    rb, rk, rid = rb[order], rk[order], rid[order]
    NB = n_buckets(D, l)
    counts = np.bincount(rb, minlength=NB)
    starts = np.concatenate([[0], np.cumsum(counts)])
    keep = counts.astype(np.int64) if threshold is not None else keep_count(counts, alpha, iProbes, rounding, kappa)
    offsets = np.concatenate([[0], np.cumsum(keep)]).astype(np.int64)
    rank = np.arange(rb.shape[0]) - starts[rb]
    sel = rank < keep[rb]
    return offsets, rid[sel].astype(np.int32), rk[sel]


def build_index(X, L, D, alpha, iProbes, seed, l=2, rounding="ceil", kappa=0, center=False,
                filter="fraction", threshold=0.0) -> Index:
    """Falconn++ index (Algorithm 1) over L tables of l concatenated cross-polytope hashes.

    kappa > 0: limit scaling; center: hash x - c (queries are hashed as given, since
    argmax x^T q = argmax (x - c)^T q, Section 3.4); filter "threshold": the global threshold
    of the theoretical LSF comparison, with threshold t > 0 given or derived from alpha.
    """
    X = np.ascontiguousarray(X, dtype=np.float32)
    n, d = X.shape
    P = padded_dim(d, D)
    S = rotation_signs(seed, L, l, P)
    idx = Index(X=X, L=L, D=D, l=l, P=P, alpha=alpha, iProbes=iProbes, seed=seed, signs=S)
    Xh = X
    if center:
        idx.center = center_vector(X)
        Xh = (X - idx.center[None, :]).astype(np.float32)
    T = None
    if filter == "threshold":
        T = (np.float32(max(0.0, float(P) * float(np.float32(threshold)))) if threshold > 0
             else lsf_threshold(alpha, D, l, P))
        idx.threshold = T
    for t in range(L):
        off, ids, keys = build_table(Xh, S[t], D, l, alpha, iProbes, rounding,
                                     0 if T is not None else kappa, T)
        idx.offsets.append(off)
        idx.ids.append(ids)
        idx.keys.append(keys)
    return idx


# ----------------------------------------------------------------------------------------------
# Query (Section 3.4 "multi-probing for querying"; Section 1 problem statement).
# ----------------------------------------------------------------------------------------------
def query_lists(index: Index, q: np.ndarray):
    """Sorted lists of one query under every (table, function): list of per-table lists."""
    q2 = np.asarray(q, dtype=np.float32).reshape(1, -1)
    return [[hash_lists(q2, index.signs[t, f], index.D) for f in range(index.l)]
            for t in range(index.L)]


def probes(index: Index, q: np.ndarray, qProbes: int, score: str = "sum") -> np.ndarray:
    """The global top-qProbes (table, bucket) of one query, best first (reading R7).

    Every (table, pair) is scored by the float32 sum of its |projections|
    (l = 1: the single |projection|) and ranked by
    (score desc, table asc, position1 asc, position2 asc).
    score "gap": the multi-probe score of plain Falconn (Section 2.2): the float32 difference
    between the pair's score and the best pair of its table (reading R17), ranked the same way.
    Returns int64 [min(qProbes, L*D^l)] of table * (2D)^l + bucket.
    """
    D, l, L = index.D, index.l, index.L
    NB = n_buckets(D, l)
    lists = query_lists(index, q)
    if l == 1:
        s = np.stack([lists[t][0].a[0] for t in range(L)])                          # [L][D]
        b = np.stack([lists[t][0].code[0] for t in range(L)]).astype(np.int64)
    else:
        s = np.stack([(lists[t][0].a[0][:, None] + lists[t][1].a[0][None, :]).astype(np.float32)
                      for t in range(L)])                                          # [L][D][D]
        b = np.stack([lists[t][0].code[0][:, None].astype(np.int64) * (2 * D)
                      + lists[t][1].code[0][None, :] for t in range(L)])
    if score == "gap":
        top = s.reshape(L, -1)[:, 0].copy()                       # position (0, 0): each table's best
        s = (s - top.reshape((L,) + (1,) * l)).astype(np.float32)
    s = s.reshape(-1)
    b = (b + (np.arange(L, dtype=np.int64) * NB).reshape((L,) + (1,) * l)).reshape(-1)
    # flat order of s is (table, pos1, pos2) lexicographic, so a stable sort on -s gives R7
    order = np.argsort(-s, kind="stable")
    qP = min(int(qProbes), s.shape[0])
    return b[order[:qP]]


def candidates(index: Index, probe_list: np.ndarray) -> np.ndarray:
    """Set union of the ids stored in the probed buckets (duplicates scored once)."""
    NB = n_buckets(index.D, index.l)
    parts = []
    for p in probe_list:
        t, bkt = divmod(int(p), NB)
        off = index.offsets[t]
        parts.append(index.ids[t][off[bkt]:off[bkt + 1]])
    if not parts:
        return np.zeros(0, dtype=np.int64)
    return np.unique(np.concatenate(parts).astype(np.int64))


def scores_f64(X: np.ndarray, q: np.ndarray, ids: np.ndarray) -> np.ndarray:
    """Inner products in float64 of exact float32 inputs."""
    return X[ids].astype(np.float64) @ np.asarray(q, dtype=np.float64)


def topk_order(scores: np.ndarray, ids: np.ndarray, k: int):
    """Reading R8: first k of (score desc, id asc), padded with (-1, -inf)."""
    order = np.lexsort((ids, -scores))[:k]
    out_i = np.full(k, -1, dtype=np.int64)
    out_s = np.full(k, -np.inf, dtype=np.float64)
    out_i[:order.shape[0]] = ids[order]
    out_s[:order.shape[0]] = scores[order]
    return out_i, out_s


def query(index: Index, Q: np.ndarray, k: int, qProbes: int, score: str = "sum"):
    """Top-k ids and float64 scores of every query, with the probe / candidate counts."""
    Q = np.atleast_2d(np.asarray(Q, dtype=np.float32))
    m = Q.shape[0]
    ids = np.empty((m, k), dtype=np.int64)
    sc = np.empty((m, k), dtype=np.float64)
    stats = np.zeros((m, 3), dtype=np.int64)    # probes, probed entries (with repeats), unique
    NB = n_buckets(index.D, index.l)
    for i in range(m):
        pl = probes(index, Q[i], qProbes, score)
        cand = candidates(index, pl)
        ent = 0
        for p in pl:
            t, bkt = divmod(int(p), NB)
            ent += int(index.offsets[t][bkt + 1] - index.offsets[t][bkt])
        stats[i] = (pl.shape[0], ent, cand.shape[0])
        s = scores_f64(index.X, Q[i], cand)
        ids[i], sc[i] = topk_order(s, cand, k)
    return ids, sc, stats


def brute_force(X: np.ndarray, Q: np.ndarray, k: int, chunk: int = 256):
    """Exact top-k over all n by (float64 score desc, id asc)."""
    X64 = np.asarray(X, dtype=np.float64)
    Q = np.atleast_2d(Q)
    n = X.shape[0]
    all_ids = np.arange(n, dtype=np.int64)
    out_i = np.empty((Q.shape[0], k), dtype=np.int64)
    out_s = np.empty((Q.shape[0], k), dtype=np.float64)
    for s0 in range(0, Q.shape[0], chunk):
        S = np.asarray(Q[s0:s0 + chunk], dtype=np.float64) @ X64.T
        for r in range(S.shape[0]):
            kk = min(k, n)
            part = np.argpartition(-S[r], kk - 1)[:kk] if kk < n else all_ids
            # widen to every score tied with the k-th so the id tie-break is exact
            kth = np.min(S[r][part])
            cand = np.nonzero(S[r] >= kth)[0]
            out_i[s0 + r], out_s[s0 + r] = topk_order(S[r][cand], cand, k)
    return out_i, out_s


def recall_at_k(found: np.ndarray, truth: np.ndarray) -> float:
    """Mean over queries of |found ∩ truth| / k (Section 4: Recall@k)."""
    k = truth.shape[1]
    hits = 0
    for f, t in zip(found, truth):
        hits += len(set(int(x) for x in f if x >= 0) & set(int(x) for x in t if x >= 0))
    return hits / (k * truth.shape[0])


# ----------------------------------------------------------------------------------------------
# Low-precision scoring stores (not in the paper): round-to-nearest-even quantisers.
# ----------------------------------------------------------------------------------------------
def bf16_bits(x: np.ndarray) -> np.ndarray:
    """float32 -> bfloat16 bit patterns, round to nearest, ties to even (finite inputs)."""
    u = np.asarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    lsb = (u >> np.uint64(16)) & np.uint64(1)
    r = (u + np.uint64(0x7FFF) + lsb) >> np.uint64(16)
    return r.astype(np.uint16)


def bf16_value(bits: np.ndarray) -> np.ndarray:
    return (np.asarray(bits, dtype=np.uint32) << np.uint32(16)).view(np.float32)


def _e4m3_table() -> np.ndarray:
    """Values of the non-negative finite OCP E4M3 codes 0x00..0x7E (bias 7, no infinities)."""
    v = np.empty(127, dtype=np.float64)
    for c in range(127):
        e, mnt = c >> 3, c & 7
        v[c] = (mnt / 8.0) * 2.0 ** -6 if e == 0 else (1.0 + mnt / 8.0) * 2.0 ** (e - 7)
    return v


_E4M3 = _e4m3_table()
E4M3_MAX = 448.0


def e4m3_bits(x: np.ndarray) -> np.ndarray:
    """float32 -> OCP E4M3 codes: nearest value, ties to the even code, magnitudes above 448 saturate."""
    x = np.asarray(x, dtype=np.float32).astype(np.float64)
    ax = np.abs(x)
    hi = np.clip(np.searchsorted(_E4M3, ax, side="left"), 0, 126)   # first value >= ax
    lo = np.maximum(hi - 1, 0)
    dlo = ax - _E4M3[lo]
    dhi = _E4M3[hi] - ax
    pick_hi = (dhi < dlo) | ((dhi == dlo) & (hi % 2 == 0))
    c = np.where(pick_hi, hi, lo)
    c = np.where(ax >= E4M3_MAX, 126, c)
    c = np.where(ax <= _E4M3[0], 0, c)
    sign = np.signbit(x)
    return (c | np.where(sign, 0x80, 0)).astype(np.uint8)


def e4m3_value(bits: np.ndarray) -> np.ndarray:
    b = np.asarray(bits, dtype=np.uint8)
    mag = _E4M3[np.minimum(b & 0x7F, 126)]
    return np.where(b & 0x80, -mag, mag).astype(np.float32)


def quantize_fp8_rows(X: np.ndarray):
    """Per-vector scale s = fl32(max|x| / 448) (1 for a zero vector); codes = E4M3(fl32(x / s))."""
    X = np.asarray(X, dtype=np.float32)
    mx = np.max(np.abs(X), axis=1).astype(np.float32)
    s = (mx / np.float32(E4M3_MAX)).astype(np.float32)
    s[mx == 0] = np.float32(1.0)
    codes = e4m3_bits((X / s[:, None]).astype(np.float32))
    return codes, s


def dequantized_store(X: np.ndarray, storage: str):
    """Exact float64 values the low-precision store represents, per element (scale applied for fp8)."""
    if storage == "fp32":
        return np.asarray(X, dtype=np.float64)
    if storage == "bf16":
        return bf16_value(bf16_bits(X)).astype(np.float64)
    if storage == "fp8":
        codes, s = quantize_fp8_rows(X)
        return e4m3_value(codes).astype(np.float64) * s.astype(np.float64)[:, None]
    raise ValueError(storage)


def simhash_bits(V: np.ndarray, signs: np.ndarray, D: int, F: int) -> np.ndarray:
    """SimHash signature (Section 4: the signs of projections already computed for the tables):
    bit g*D + i is 1 when projection i of hash function g (in table-major, function-minor order)
    is negative (reading R18). Returns bool [n][F*D]."""
    L, l = signs.shape[:2]
    V = np.asarray(V, dtype=np.float32)
    out = np.zeros((V.shape[0], F * D), dtype=bool)
    for g in range(F):
        t, f = divmod(g, l)
        out[:, g * D:(g + 1) * D] = rotate(V, signs[t, f], D) < np.float32(0.0)
    return out


def simhash_words(bits: np.ndarray) -> np.ndarray:
    """Pack signature bits little-endian into 32-bit words: bit b -> word b // 32, bit b % 32."""
    n, nb = bits.shape
    w = (nb + 31) // 32
    padded = np.zeros((n, w * 32), dtype=np.uint64)
    padded[:, :nb] = bits
    weights = (np.uint64(1) << np.arange(32, dtype=np.uint64))
    return (padded.reshape(n, w, 32) * weights).sum(axis=2).astype(np.uint32)


def simhash_score(sig_x: np.ndarray, sig_q: np.ndarray) -> np.ndarray:
    """Approximate score of SimHash: bits - 2 * Hamming distance (a float, exact)."""
    ham = np.count_nonzero(sig_x != sig_q[None, :], axis=1)
    return (sig_x.shape[1] - 2 * ham).astype(np.float64)


def query_reranked(index: Index, Q: np.ndarray, k: int, qProbes: int, R: int, storage: str,
                   store: np.ndarray | None = None, simhash_functions: int = 0):
    """Low-precision form: approximate scores on the store, short list of R, exact float64 rerank.

    Short list = first R candidates by (approximate score desc, id asc); the final answer
    is the top-k of the short list by exact score (reading R8).
    """
    Q = np.atleast_2d(np.asarray(Q, dtype=np.float32))
    if storage == "simhash":
        F = simhash_functions
        qsig = simhash_bits(Q, index.signs, index.D, F)
    m = Q.shape[0]
    ids = np.empty((m, k), dtype=np.int64)
    sc = np.empty((m, k), dtype=np.float64)
    short = np.empty((m, R), dtype=np.int64)
    for i in range(m):
        pl = probes(index, Q[i], qProbes)
        cand = candidates(index, pl)
        # the store's rows of the candidates (every quantiser works row by row, so quantising
        # only these rows gives the values of the whole store)
        if store is not None:
            rows = store[cand]
        elif storage == "simhash":
            rows = simhash_bits(index.X[cand], index.signs, index.D, F)
        else:
            rows = dequantized_store(index.X[cand], storage)
        if storage == "simhash":
            approx = simhash_score(rows, qsig[i])
        else:
            approx = rows @ Q[i].astype(np.float64)
        sl, _ = topk_order(approx, cand, R)
        short[i] = sl
        sl = sl[sl >= 0]
        ex = scores_f64(index.X, Q[i], sl)
        ids[i], sc[i] = topk_order(ex, sl, k)
    return ids, sc, short
