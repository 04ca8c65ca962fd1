"""Seeded synthetic workloads for the Falconn++ hot path.

This module only draws random numbers and normalises vectors. It holds none of
the method's arithmetic (no rotation, hashing, filtering or scoring), so both
the CPU oracle and the GPU path may take their inputs from it.

The paper evaluates on Glove200, Glove300 and NYTimes (Section 4, "Data sets"
table). Those corpora are not available here; the clustered unit-sphere
mixtures below stand in for them. They reproduce the regime the introduction
describes, where nearest-neighbour distance gaps are tiny: in the n=1M, d=128
workload two points of one cluster have cosine about 0.917.

All draws use ``numpy.random.Generator(PCG64(seed))`` in a fixed order, in
float64, and vectors are normalised in float64 before the cast to float32.
"""
from __future__ import annotations

import dataclasses

import numpy as np

__all__ = [
    "Workload",
    "gaussian_sphere",
    "clustered_sphere",
    "workload",
    "WORKLOADS",
]


@dataclasses.dataclass
class Workload:
    """One synthetic workload: data X (n x d float32), queries Q (m x d float32) and index parameters."""

    name: str
    X: np.ndarray
    Q: np.ndarray
    L: int
    D: int
    l: int
    alpha: float
    iProbes: int
    k: int
    qprobes_per_table: tuple
    seed: int


def _normalise_rows(A: np.ndarray) -> np.ndarray:
    nrm = np.sqrt(np.einsum("ij,ij->i", A, A))
    nrm[nrm == 0.0] = 1.0
    return (A / nrm[:, None]).astype(np.float32)


def gaussian_sphere(n: int, d: int, m: int, noise: float, seed: int):
    """i.i.d. N(0, I_d) points on the sphere; queries are m distinct data points plus N(0, noise^2) noise.

    Draw order: X (n x d), then the m query indices (without replacement), then the m x d noise.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    X64 = rng.standard_normal((n, d))
    X = _normalise_rows(X64)
    idx = rng.choice(n, size=m, replace=False)
    Q64 = X64[idx] / np.linalg.norm(X64[idx], axis=1, keepdims=True)
    Q64 = Q64 + rng.normal(0.0, noise, size=(m, d))
    Q = _normalise_rows(Q64)
    return X, Q


def clustered_sphere(n: int, d: int, m: int, n_centers: int, spread: float, seed: int,
                     chunk: int = 1 << 20):
    """Gaussian mixture on the sphere: centres ~ N(0, I_d) normalised; x = c_label + N(0, spread^2/d I_d), normalised.

    Draw order: centres (n_centers x d), data labels (n), data noise in chunks of
    ``chunk`` rows, query labels (m), query noise (m x d).
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    C = rng.standard_normal((n_centers, d))
    C /= np.linalg.norm(C, axis=1, keepdims=True)
    labels = rng.integers(0, n_centers, size=n)
    sd = spread / np.sqrt(d)
    X = np.empty((n, d), dtype=np.float32)
    for s in range(0, n, chunk):
        e = min(n, s + chunk)
        X[s:e] = _normalise_rows(C[labels[s:e]] + rng.normal(0.0, sd, size=(e - s, d)))
    qlab = rng.integers(0, n_centers, size=m)
    Q = _normalise_rows(C[qlab] + rng.normal(0.0, sd, size=(m, d)))
    return X, Q


# Parameters per workload. qprobes_per_table is the sweep of probes per table;
# the query call receives the total over all tables (per-table value x L).
WORKLOADS = {
    # n=10k, d=64 Gaussian; L=10 tables of one cross-polytope hash, D=64.
    "c1_gauss_10k_d64": dict(kind="gauss", n=10_000, d=64, m=100, noise=0.05, seed=0,
                             L=10, D=64, l=1, alpha=0.5, iProbes=1, k=10, qpt=(4,)),
    # n=1M, d=128, 1000 clusters, spread 0.3; L=100 tables of two concatenated hashes, D=128.
    "c2_cluster_1m_d128": dict(kind="cluster", n=1_000_000, d=128, m=10_000, centers=1000,
                               spread=0.3, seed=0, L=100, D=128, l=2, alpha=0.3, iProbes=3,
                               k=10, qpt=(10, 20, 50, 100, 200)),
    # the headline shape with four times the points and clusters (n=4M, 4000 clusters of about
    # 1000 points): its BF16 store (1 GB) is four times the 256 MB last-level cache of the GPU
    "c2x4_cluster_4m_d128": dict(kind="cluster", n=4_000_000, d=128, m=10_000, centers=4000,
                                 spread=0.3, seed=0, L=100, D=128, l=2, alpha=0.3, iProbes=3,
                                 k=10, qpt=(10, 20, 50, 100, 200)),
    # n=1M, d=300, 2000 clusters, spread 0.4; L=128, D=256 (hash pads d to 512).
    "c3_cluster_1m_d300": dict(kind="cluster", n=1_000_000, d=300, m=10_000, centers=2000,
                               spread=0.4, seed=0, L=128, D=256, l=2, alpha=0.2, iProbes=3,
                               k=10, qpt=(10, 20, 50, 100, 200)),
    # n=10M, d=96, 10000 clusters, spread 0.35; L=64, D=256.
    "c5_cluster_10m_d96": dict(kind="cluster", n=10_000_000, d=96, m=100_000, centers=10_000,
                               spread=0.35, seed=0, L=64, D=256, l=2, alpha=0.1, iProbes=2,
                               k=10, qpt=(100,)),
}


def workload(name: str, n: int | None = None, m: int | None = None, seed: int | None = None) -> Workload:
    """Materialise a named workload; ``n``/``m``/``seed`` override the defaults (for scaled-down tests)."""
    p = dict(WORKLOADS[name])
    n = p["n"] if n is None else n
    m = p["m"] if m is None else m
    seed = p["seed"] if seed is None else seed
    if p["kind"] == "gauss":
        X, Q = gaussian_sphere(n, p["d"], m, p["noise"], seed)
    else:
        X, Q = clustered_sphere(n, p["d"], m, p["centers"], p["spread"], seed)
    return Workload(name=name, X=X, Q=Q, L=p["L"], D=p["D"], l=p["l"], alpha=p["alpha"],
                    iProbes=p["iProbes"], k=p["k"], qprobes_per_table=tuple(p["qpt"]), seed=seed)
