"""Host-side logic of bench.py (no GPU): the qProbes search, the sustained-rate search, the
algorithmic byte count and the guard on the profiled traffic figure."""
import hashlib
import json
import os

import numpy as np
import pytest

import bench


@pytest.mark.parametrize("need", [1, 4, 9, 10, 11, 19, 20, 27, 49, 50, 51, 777, 20000])
def test_smallest_qprobes_finds_the_first_reaching_total(need):
    seen = []

    def rec(qp):
        seen.append(qp)
        return 0.95 if qp >= need else 0.5
    assert bench.smallest_qprobes(rec) == need
    # the grid up to the first value reaching the target, then a bisection of that interval
    grid = [g for g in bench.QP_SWEEP if g < need] + [min(g for g in bench.QP_SWEEP if g >= need)]
    assert seen[:len(grid)] == grid
    assert len(seen) - len(grid) <= int(np.ceil(np.log2(max(2, grid[-1] - (grid[-2] if len(grid) > 1 else 0)))))


def test_smallest_qprobes_none_when_the_target_is_never_reached():
    assert bench.smallest_qprobes(lambda qp: 0.5) is None


def test_smallest_qprobes_on_a_recall_curve():
    # a recall curve that rises with qProbes (as nested probe sets make it)
    curve = lambda qp: 1.0 - np.exp(-qp / 12.0)
    got = bench.smallest_qprobes(curve)
    assert curve(got) >= 0.9 and curve(got - 1) < 0.9


def test_sustained_search_brackets_the_capacity():
    limit = 1.13e6

    def run(rate):
        return {"sustained": rate <= limit, "rate": rate}
    best, runs = bench.sustained_search(run, 1e6)
    assert best["rate"] <= limit
    assert limit - best["rate"] <= 0.5 * 1e6 / 2 ** 6 + 1
    assert runs[0]["rate"] == pytest.approx(0.8e6)


def test_sustained_search_halves_below_the_first_point():
    best, runs = bench.sustained_search(lambda r: {"sustained": r <= 0.3e6, "rate": r}, 1e6)
    assert best is not None and best["rate"] <= 0.3e6
    assert [round(r["rate"]) for r in runs[:3]] == [800000, 400000, 200000]


def test_algorithmic_bytes():
    st = np.array([[27, 1791, 863], [10, 100, 50]], dtype=np.int64)   # probes, entries, unique
    d, k, R = 128, 10, 100
    assert bench.algorithmic_bytes(st, d, "fp32", k, R) == 8 * 37 + 4 * 1891 + 512 * 913 + 80 * 2
    assert bench.algorithmic_bytes(st, d, "bf16", k, R) == 8 * 37 + 4 * 1891 + 256 * 913 + 400 * 2
    assert bench.algorithmic_bytes(st, d, "fp8", k, R) == 8 * 37 + 4 * 1891 + 132 * 913 + 400 * 2


def test_traffic_figure_requires_the_profiled_source_and_qprobes():
    rec = json.load(open(os.path.join(bench.ROOT, "profiles", "score_kernel_traffic.json")))
    src = os.path.join(bench.ROOT, "paper_2206_01382_amd", "csrc", "score.hip")
    same_source = hashlib.sha256(open(src, "rb").read()).hexdigest() == rec["score_hip_sha256"]
    got = bench.traffic_per_call({"qprobes": rec["qprobes"]})
    assert got == (rec["hbm_bytes_per_call"] if same_source else None)
    assert bench.traffic_per_call({"qprobes": rec["qprobes"] + 1}) is None
