"""Writes the oracle's expected values for the full-size parity tests (test infrastructure).

Calls only ``oracle/`` and ``synthdata/``: every table is built by ``oracle.falconn.build_table``
and every query answered by ``oracle.falconn.query`` / ``query_reranked`` on the oracle's own
index, in a process pool (tables in parallel, then query shards in parallel). Nothing here reads
the GPU library.

    python tests/golden/make_fullsize_oracle.py c2     # -> tests/golden/c2_full_oracle.json
    python tests/golden/make_fullsize_oracle.py c5     # -> tests/golden/c5_shape_oracle.json

c2: the headline index (n = 1M, d = 128, L = 100, D = 128, l = 2, alpha = 0.3, iProbes = 3,
    seed 42) and 200 of its 10,000 queries (every 50th), at 27 probes in total (the smallest
    total reaching recall@10 0.9 on these queries' batch), at 50 and at 50 per table, plus the
    BF16 and FP8 short lists of 100 reranked in FP64 at 27 probes.
c5: the large workload's data and hash shape (n = 10M, d = 96 -> P = 256, D = 256, l = 2,
    alpha = 0.1, iProbes = 2, seed 42) with 4 of its 64 tables, and 200 of its 100,000 queries
    (every 500th) at 100 probes per table (400 in total), FP32 and FP8 with the rerank of 100.

Each table is recorded as the SHA-256 of its CSR (offsets as little-endian int64 starting at
0, then ids as little-endian int32), its size and its largest bucket; each probe set (at the
first probe count) as the SHA-256 of its sorted entries; results as ids and float64 scores.
"""
from __future__ import annotations

import hashlib
import json
import multiprocessing as mp
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import synthdata  # noqa: E402
from oracle import falconn as O  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))

SPECS = {
    "c2": dict(workload="c2_cluster_1m_d128", L=100, seed=42, q_stride=50,
               qprobes=(27, 50, 5000), rerank=dict(qprobes=27, R=100, stores=("bf16", "fp8")),
               probes_at=27, out="c2_full_oracle.json"),
    "c5": dict(workload="c5_cluster_10m_d96", L=4, seed=42, q_stride=500,
               qprobes=(400,), rerank=dict(qprobes=400, R=100, stores=("fp8",)),
               probes_at=400, out="c5_shape_oracle.json"),
}

_G = {}   # shared with forked workers


def table_digest(offsets: np.ndarray, ids: np.ndarray) -> str:
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(offsets, dtype="<i8").tobytes())
    h.update(np.ascontiguousarray(ids, dtype="<i4").tobytes())
    return h.hexdigest()


def probe_digest(probes: np.ndarray) -> str:
    """First 16 hex digits of the SHA-256 of a probe set (sorted, little-endian int64)."""
    return hashlib.sha256(np.sort(np.asarray(probes, dtype="<i8")).tobytes()).hexdigest()[:16]


def _build(t):
    w, S = _G["w"], _G["S"]
    t0 = time.perf_counter()
    off, ids, _ = O.build_table(w.X, S[t], w.D, w.l, w.alpha, w.iProbes)
    print(f"  table {t}: {len(ids)} ids in {time.perf_counter() - t0:.0f}s", flush=True)
    return t, off, ids


def _answer(job):
    kind, qp, rows = job
    idx, Q = _G["idx"], _G["Q"]
    if kind == "fp32":
        ids, sc, st = O.query(idx, Q[rows], 10, qp)
        pr = [probe_digest(O.probes(idx, Q[r], qp)) for r in rows] if qp == _G["probes_at"] else None
        return kind, qp, rows, ids, sc, st, pr
    ids, sc, _ = O.query_reranked(idx, Q[rows], 10, qp, R=_G["R"], storage=kind)
    return kind, qp, rows, ids, sc, None, None


def main(name: str, workers: int):
    spec = SPECS[name]
    t0 = time.perf_counter()
    w = synthdata.workload(spec["workload"])
    L = spec["L"]
    P = O.padded_dim(w.X.shape[1], w.D)
    S = O.rotation_signs(spec["seed"], L, w.l, P)
    print(f"{name}: data {w.X.shape} in {time.perf_counter() - t0:.0f}s", flush=True)
    _G.update(w=w, S=S)
    ctx = mp.get_context("fork")
    with ctx.Pool(workers) as pool:
        built = sorted(pool.map(_build, range(L), chunksize=1))
    idx = O.Index(X=w.X, L=L, D=w.D, l=w.l, P=P, alpha=w.alpha, iProbes=w.iProbes, seed=spec["seed"],
                  signs=S, offsets=[b[1] for b in built], ids=[b[2] for b in built])
    tables = [dict(sha256=table_digest(off, ids), size=int(len(ids)), max_bucket=int(np.max(np.diff(off))))
              for _, off, ids in built]
    print(f"{name}: tables in {time.perf_counter() - t0:.0f}s", flush=True)
    rows = np.arange(0, w.Q.shape[0], spec["q_stride"], dtype=np.int64)
    _G.update(idx=idx, Q=w.Q, probes_at=spec["probes_at"], R=spec["rerank"]["R"])
    shards = np.array_split(rows, workers * 2)
    jobs = [("fp32", qp, s) for qp in spec["qprobes"] for s in shards]
    jobs += [(st, spec["rerank"]["qprobes"], s) for st in spec["rerank"]["stores"] for s in shards]
    out = {"workload": spec["workload"], "n": int(w.X.shape[0]), "d": int(w.X.shape[1]), "L": L,
           "D": w.D, "l": w.l, "alpha": w.alpha, "iProbes": w.iProbes, "seed": spec["seed"], "k": 10,
           "queries": rows.tolist(), "tables": tables, "fp32": {}, "rerank": {}}
    res = {}
    with ctx.Pool(workers) as pool:
        for kind, qp, rws, ids, sc, extra, pr in pool.imap_unordered(_answer, jobs):
            res.setdefault((kind, qp), []).append((rws, ids, sc, extra, pr))
    for (kind, qp), parts in res.items():
        parts.sort(key=lambda p: int(p[0][0]))
        ids = np.concatenate([p[1] for p in parts])
        sc = np.concatenate([p[2] for p in parts])
        rec = {"ids": ids.tolist(), "scores": [[float(v) for v in r] for r in sc]}
        if kind == "fp32":
            rec["stats"] = np.concatenate([p[3] for p in parts]).tolist()
            if parts[0][4] is not None:
                rec["probe_sha256"] = [pl for p in parts for pl in p[4]]
            out["fp32"][str(qp)] = rec
        else:
            rec["qProbes"] = qp
            rec["R"] = spec["rerank"]["R"]
            out["rerank"][kind] = rec
    path = os.path.join(HERE, spec["out"])
    with open(path, "w") as f:
        json.dump(out, f, separators=(",", ":"))
    print(f"{name}: wrote {path} in {time.perf_counter() - t0:.0f}s", flush=True)


if __name__ == "__main__":
    main(sys.argv[1], int(sys.argv[2]) if len(sys.argv) > 2 else min(8, os.cpu_count() or 1))
