"""Comparison rule of the GPU path against the oracle (shared by the GPU test modules).

Scores: |s32 - s64| <= 1e-6 |s64| where |s64| >= 0.1, else <= 1e-6 sum_j |q_j x_j| (relative
error is undefined near zero), with s64 the float64 dot product of the exact float32 inputs (of
the dequantised rows for a low-precision store's approximate scores). The bound does not depend
on how the kernel lays out its reduction.

Ids: identical, except where the GPU's id and the oracle's id at a position have float64 scores
within twice that bound of each other (an adjudicated near-tie). Every such position is counted
per test, and the counts are printed at the end of the session.
"""
from __future__ import annotations

import os

import numpy as np

# test id -> [adjudicated positions, compared result positions]
SWAPS: dict[str, list[int]] = {}


def score_tol(s64, sabs):
    s64 = np.asarray(s64, dtype=np.float64)
    return np.where(np.abs(s64) >= 0.1, 1e-6 * np.abs(s64), 1e-6 * np.asarray(sabs, dtype=np.float64))


def _label(label):
    if label:
        return label
    cur = os.environ.get("PYTEST_CURRENT_TEST", "?")
    return cur.rsplit(" ", 1)[0]


def check_topk(X, Q, gi, gs, oi_ids, oi_sc, k=None, d=None, store=None, label=None):
    """GPU top-k (gi, gs) against the oracle's (oi_ids, oi_sc) for the rows of Q; X holds the
    values the scores are defined on. Returns the number of adjudicated positions."""
    gi = np.asarray(gi).astype(np.int64)
    oi_ids = np.asarray(oi_ids).astype(np.int64)
    swaps = 0
    X64 = np.asarray(X, dtype=np.float64)
    for r in range(Q.shape[0]):
        q = np.asarray(Q[r], dtype=np.float64)
        valid = gi[r] >= 0
        assert np.array_equal(valid, oi_ids[r] >= 0), (r, gi[r], oi_ids[r])
        ids = gi[r][valid]
        assert len(set(ids.tolist())) == len(ids)
        s64 = X64[ids] @ q
        sabs = np.abs(X64[ids] * q).sum(1)
        tol = score_tol(s64, sabs)
        err = np.abs(np.asarray(gs[r], dtype=np.float64)[valid] - s64)
        assert np.all(err <= tol), (r, float(np.max(err / np.maximum(tol, 1e-300))))
        assert np.all(np.isneginf(np.asarray(gs[r])[~valid]))
        if not np.array_equal(gi[r], oi_ids[r]):
            # the oracle's score at each differing position must be within twice the bound of
            # the score of the id the GPU returned there
            diff = gi[r] != oi_ids[r]
            osc = np.asarray(oi_sc[r], dtype=np.float64)
            assert np.all(np.abs(s64 - osc[valid]) <= 2 * tol), (r, gi[r], oi_ids[r])
            swaps += int(np.sum(diff))
    rec = SWAPS.setdefault(_label(label), [0, 0])
    rec[0] += swaps
    rec[1] += int(np.asarray(gi).size)
    return swaps


def swap_budget(results: int) -> int:
    """Adjudicated positions allowed in a comparison of `results` positions: 0.1%, at least 2."""
    return max(2, results // 1000)
