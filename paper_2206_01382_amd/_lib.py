"""ctypes binding of libfpp (include/fpp.h): the same entry points, argument marshalling only.

Tensors passed to the library must be contiguous tensors on the current HIP device; the
library receives their data pointers and the current torch stream. Every step of the
Falconn++ path runs in the library's HIP kernels; nothing here computes.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfpp.so")

FPP_OK = 0
FPP_EINVAL = -1
FPP_ENOMEM = -2
FPP_EHIP = -3
FPP_ECAPACITY = -4
FPP_ESTATE = -5

FPP_STORE_FP32 = 0
FPP_STORE_BF16 = 1
FPP_STORE_FP8 = 2
FPP_STORE_SIMHASH = 3
STORES = {"fp32": FPP_STORE_FP32, "bf16": FPP_STORE_BF16, "fp8": FPP_STORE_FP8, "simhash": FPP_STORE_SIMHASH}

c_i32, c_i64, c_u64, c_f32, c_vp = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_float, ctypes.c_void_p


FPP_FILTER_FRACTION = 0
FPP_FILTER_THRESHOLD = 1
FILTERS = {"fraction": FPP_FILTER_FRACTION, "threshold": FPP_FILTER_THRESHOLD}


class fpp_build_opts(ctypes.Structure):
    _fields_ = [("l", c_i32), ("stores", c_i32), ("keep_rounding", c_i32), ("tables_per_pass", c_i32),
                ("kappa", c_i32), ("center", c_i32), ("filter", c_i32), ("threshold", c_f32),
                ("simhash_functions", c_i32)]


FPP_PROBE_SUM = 0
FPP_PROBE_GAP = 1
PROBE_SCORES = {"sum": FPP_PROBE_SUM, "gap": FPP_PROBE_GAP}


class fpp_query_opts(ctypes.Structure):
    _fields_ = [("store", c_i32), ("rerank_R", c_i32), ("stats", c_vp), ("stage_ms", c_vp),
                ("probe_score", c_i32)]


class fpp_index_info(ctypes.Structure):
    _fields_ = [("n", c_i64), ("d", c_i32), ("L", c_i32), ("D", c_i32), ("l", c_i32), ("P", c_i32),
                ("iProbes", c_i32), ("stores", c_i32), ("alpha", c_f32), ("seed", c_u64),
                ("buckets_per_table", c_i64), ("total_ids", c_i64), ("max_bucket", c_i64),
                ("device_bytes", c_i64), ("build_ms", ctypes.c_double), ("kappa", c_i32),
                ("centered", c_i32), ("filter", c_i32), ("threshold", c_f32), ("simhash_bits", c_i32),
                ("overflow_sets", c_i32)]


class fpp_server_opts(ctypes.Structure):
    _fields_ = [("scratch_bytes", c_i64), ("n_streams", c_i32), ("max_batch", c_i32),
                ("store", c_i32), ("rerank_R", c_i32), ("probe_score", c_i32)]


class fpp_server_stats(ctypes.Structure):
    _fields_ = [("submitted", c_i64), ("completed", c_i64), ("failed", c_i64), ("batches", c_i64),
                ("queries", c_i64), ("max_inflight_batches", c_i64), ("scratch_high_water", c_i64)]


# name -> (restype, argtypes)
SIGNATURES = {
    "fpp_default_build_opts": (None, [ctypes.POINTER(fpp_build_opts)]),
    "fpp_build_index": (c_i32, [c_vp, c_i64, c_i32, c_i32, c_i32, c_f32, c_i32, c_u64, ctypes.POINTER(c_vp)]),
    "fpp_build_index_ex": (c_i32, [c_vp, c_i64, c_i32, c_i32, c_i32, c_f32, c_i32, c_u64,
                                   ctypes.POINTER(fpp_build_opts), c_vp, ctypes.POINTER(c_vp)]),
    "fpp_free_index": (None, [c_vp]),
    "fpp_default_query_opts": (None, [ctypes.POINTER(fpp_query_opts)]),
    "fpp_query": (c_i32, [c_vp, c_vp, c_i64, c_i32, c_i32, c_vp, c_vp, c_vp]),
    "fpp_query_ex": (c_i32, [c_vp, c_vp, c_i64, c_i32, c_i32, ctypes.POINTER(fpp_query_opts), c_vp, c_vp, c_vp]),
    "fpp_query_ex_noalloc": (c_i32, [c_vp, c_vp, c_i64, c_i32, c_i32, ctypes.POINTER(fpp_query_opts), c_vp, c_vp, c_vp]),
    "fpp_query_batch": (c_i32, [c_vp, c_vp, c_i64, c_vp, c_vp, ctypes.POINTER(fpp_query_opts), c_vp, c_vp, c_vp]),
    "fpp_query_workspace_bytes": (c_i64, [c_vp, c_i64, c_i32, c_i32, ctypes.POINTER(fpp_query_opts)]),
    "fpp_index_get_info": (c_i32, [c_vp, ctypes.POINTER(fpp_index_info)]),
    "fpp_index_table_sizes": (c_i32, [c_vp, c_vp]),
    "fpp_last_error": (ctypes.c_char_p, []),
    "fpp_version": (ctypes.c_char_p, []),
    "fpp_default_server_opts": (None, [ctypes.POINTER(fpp_server_opts)]),
    "fpp_server_create": (c_i32, [c_vp, ctypes.POINTER(fpp_server_opts), ctypes.POINTER(c_vp)]),
    "fpp_server_submit": (c_i32, [c_vp, c_vp, c_i32, c_i32, c_i32, c_vp, c_vp, ctypes.POINTER(c_i64)]),
    "fpp_server_replay": (c_i32, [c_vp, c_vp, c_i64, c_i64, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp]),
    "fpp_server_poll": (c_i32, [c_vp, c_i64, ctypes.POINTER(c_i32), ctypes.POINTER(c_i64), ctypes.POINTER(c_i64)]),
    "fpp_server_wait": (c_i32, [c_vp, c_i64, c_i64, ctypes.POINTER(c_i32), ctypes.POINTER(c_i64),
                                ctypes.POINTER(c_i64)]),
    "fpp_server_get_stats": (c_i32, [c_vp, ctypes.POINTER(fpp_server_stats)]),
    "fpp_server_debug_fail_batches": (c_i32, [c_vp, c_i32]),
    "fpp_server_destroy": (None, [c_vp]),
    "fpp_debug_signs": (c_i32, [c_vp, c_vp]),
    "fpp_debug_query_lists": (c_i32, [c_vp, c_vp, c_i64, c_vp, c_vp, c_vp]),
    "fpp_debug_query_list_prefix": (c_i32, [c_vp, c_vp, c_i64, c_i32, c_vp, c_vp, c_vp]),
    "fpp_debug_build_records": (c_i32, [c_vp, c_i32, c_vp, c_vp, c_vp]),
    "fpp_debug_export_table": (c_i32, [c_vp, c_i32, c_vp, c_vp]),
    "fpp_debug_probes": (c_i32, [c_vp, c_vp, c_i64, c_i32, c_i32, c_vp, c_vp]),
    "fpp_debug_export_store": (c_i32, [c_vp, c_i32, c_vp, c_vp, c_vp]),
    "fpp_debug_center": (c_i32, [c_vp, c_vp]),
    "fpp_debug_set_partition_threshold": (c_i32, [c_vp, c_i64, c_i32]),
    "fpp_debug_set_rerank_cut": (c_i32, [c_vp, c_i32]),
    "fpp_normal_quantile": (ctypes.c_double, [ctypes.c_double]),
}

_LIB = None


class FppError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"fpp error {code}: {msg}")
        self.code = code


def lib():
    """The loaded library. Raises if libfpp.so has not been built: there is no fallback path."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2206_01382_amd.build_lib.build()")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)   # AttributeError: the library lacks a declared entry point
            f.restype = res
            f.argtypes = args
        _LIB = L
    return _LIB


def _check(rc: int):
    if rc != FPP_OK:
        raise FppError(rc, lib().fpp_last_error().decode())


def _torch():
    import torch
    return torch


def _dev(t, dtype, name):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a GPU tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return c_vp(t.data_ptr())


def _stream(stream):
    torch = _torch()
    s = torch.cuda.current_stream() if stream is None else stream
    return c_vp(s.cuda_stream)


# ------------------------------------------------------------------------------------------------
def fpp_build_index(X, L: int, D: int, alpha: float, iProbes: int, seed: int, *, l: int = 2,
                    stores=(), keep_rounding: int = 0, tables_per_pass: int = 0, kappa: int = 0,
                    center: bool = False, filter: str = "fraction", threshold: float = 0.0,
                    simhash_functions: int = 0, stream=None) -> c_vp:
    """Build an index over X (GPU float32 [n][d]); returns the opaque handle."""
    torch = _torch()
    xp = _dev(X, torch.float32, "X")
    o = fpp_build_opts(l, sum(1 << STORES[s] for s in stores), keep_rounding, tables_per_pass,
                       kappa, int(bool(center)), FILTERS[filter], threshold, simhash_functions)
    h = c_vp()
    _check(lib().fpp_build_index_ex(xp, X.shape[0], X.shape[1], L, D, alpha, iProbes, seed & (2 ** 64 - 1),
                                    ctypes.byref(o), _stream(stream), ctypes.byref(h)))
    return h


def fpp_free_index(h):
    if h is not None and h.value:
        lib().fpp_free_index(h)


def fpp_query(h, Q, k: int, qProbes: int, *, store: str = "fp32", rerank_R: int = 0, stats: bool = False,
              stream=None, out=None, stage_ms=None, probe_score: str = "sum"):
    """Top-k of every row of Q (GPU float32 [m][d]) -> (ids int32 [m][k], scores float32 [m][k][, stats]).

    ``stage_ms``: optional numpy float64 array of 4 that receives per-stage milliseconds
    (hashing, probe selection, gather/score/top-k, rerank); the call then synchronises.
    """
    torch = _torch()
    m = Q.shape[0]
    qp = _dev(Q, torch.float32, "Q") if m else c_vp(0)
    if out is None:
        ids = torch.empty((m, k), dtype=torch.int32, device=Q.device)
        sc = torch.empty((m, k), dtype=torch.float32, device=Q.device)
    else:
        ids, sc = out
    st = torch.empty((m, 3), dtype=torch.int64, device=Q.device) if stats else None
    if stage_ms is not None and (stage_ms.dtype != np.float64 or stage_ms.shape != (4,)):
        raise ValueError("stage_ms must be a float64 array of 4")
    o = fpp_query_opts(STORES[store], rerank_R, c_vp(st.data_ptr()) if stats and m else None,
                       stage_ms.ctypes.data_as(c_vp) if stage_ms is not None else None,
                       PROBE_SCORES[probe_score])
    _check(lib().fpp_query_ex(h, qp, m, k, qProbes, ctypes.byref(o),
                              c_vp(ids.data_ptr()) if m else c_vp(0), c_vp(sc.data_ptr()) if m else c_vp(0),
                              _stream(stream)))
    return (ids, sc, st) if stats else (ids, sc)


def fpp_query_ex_noalloc(h, Q, k: int, qProbes: int, *, store: str = "fp32", rerank_R: int = 0,
                         stats: bool = False, stream=None, probe_score: str = "sum"):
    """fpp_query without allocation inside the library (static device scratch; overlapping calls
    on one device race). The output tensors are allocated here, by the caller of the C ABI."""
    torch = _torch()
    m = Q.shape[0]
    qp = _dev(Q, torch.float32, "Q") if m else c_vp(0)
    ids = torch.empty((m, k), dtype=torch.int32, device=Q.device)
    sc = torch.empty((m, k), dtype=torch.float32, device=Q.device)
    st = torch.empty((m, 3), dtype=torch.int64, device=Q.device) if stats else None
    o = fpp_query_opts(STORES[store], rerank_R, c_vp(st.data_ptr()) if stats and m else None, None,
                       PROBE_SCORES[probe_score])
    _check(lib().fpp_query_ex_noalloc(h, qp, m, k, qProbes, ctypes.byref(o),
                                      c_vp(ids.data_ptr()) if m else c_vp(0),
                                      c_vp(sc.data_ptr()) if m else c_vp(0), _stream(stream)))
    return (ids, sc, st) if stats else (ids, sc)


def fpp_query_batch(h, Q, k, qProbes, *, store: str = "fp32", rerank_R: int = 0, stats: bool = False,
                    stream=None, probe_score: str = "sum"):
    """Mixed batch: per-query k and qProbes (sequences); results packed in query order."""
    torch = _torch()
    m = Q.shape[0]
    ka = np.ascontiguousarray(np.asarray(k, dtype=np.int32))
    pa = np.ascontiguousarray(np.asarray(qProbes, dtype=np.int32))
    if ka.shape != (m,) or pa.shape != (m,):
        raise ValueError("k and qProbes need one entry per query")
    tot = int(ka.sum())
    ids = torch.empty(tot, dtype=torch.int32, device=Q.device)
    sc = torch.empty(tot, dtype=torch.float32, device=Q.device)
    st = torch.empty((m, 3), dtype=torch.int64, device=Q.device) if stats else None
    o = fpp_query_opts(STORES[store], rerank_R, c_vp(st.data_ptr()) if stats and m else None, None,
                       PROBE_SCORES[probe_score])
    _check(lib().fpp_query_batch(h, _dev(Q, torch.float32, "Q") if m else c_vp(0), m,
                                 ka.ctypes.data_as(c_vp), pa.ctypes.data_as(c_vp), ctypes.byref(o),
                                 c_vp(ids.data_ptr()) if tot else c_vp(0),
                                 c_vp(sc.data_ptr()) if tot else c_vp(0), _stream(stream)))
    return (ids, sc, st) if stats else (ids, sc)


def fpp_query_workspace_bytes(h, m: int, k_max: int, qprobes_max: int, store: str = "fp32", rerank_R: int = 0):
    o = fpp_query_opts(STORES[store], rerank_R, None, None, FPP_PROBE_SUM)
    return int(lib().fpp_query_workspace_bytes(h, m, k_max, qprobes_max, ctypes.byref(o)))


def fpp_index_get_info(h) -> dict:
    inf = fpp_index_info()
    _check(lib().fpp_index_get_info(h, ctypes.byref(inf)))
    return {name: getattr(inf, name) for name, _ in fpp_index_info._fields_}


def fpp_index_table_sizes(h) -> np.ndarray:
    L = fpp_index_get_info(h)["L"]
    out = np.zeros(L, dtype=np.int64)
    _check(lib().fpp_index_table_sizes(h, out.ctypes.data_as(c_vp)))
    return out


def fpp_last_error() -> str:
    return lib().fpp_last_error().decode()


def fpp_version() -> str:
    return lib().fpp_version().decode()


# ------------------------------------------------------------------------------------------------
def fpp_debug_signs(h) -> np.ndarray:
    inf = fpp_index_get_info(h)
    out = np.zeros((inf["L"], inf["l"], 3, inf["P"]), dtype=np.int8)
    _check(lib().fpp_debug_signs(h, out.ctypes.data_as(c_vp)))
    return out


def fpp_debug_query_lists(h, V, stream=None, W=None):
    """Sorted query hash lists [m][L][l][D]; with W, only positions [0, W) are defined."""
    torch = _torch()
    inf = fpp_index_get_info(h)
    m = V.shape[0]
    a = torch.empty((m, inf["L"], inf["l"], inf["D"]), dtype=torch.float32, device=V.device)
    c = torch.empty((m, inf["L"], inf["l"], inf["D"]), dtype=torch.int32, device=V.device)
    Vp = _dev(V, torch.float32, "V")
    if W is None:
        _check(lib().fpp_debug_query_lists(h, Vp, m, c_vp(a.data_ptr()), c_vp(c.data_ptr()),
                                           _stream(stream)))
    else:
        _check(lib().fpp_debug_query_list_prefix(h, Vp, m, int(W), c_vp(a.data_ptr()),
                                                 c_vp(c.data_ptr()), _stream(stream)))
    return a, c


def fpp_debug_center(h) -> np.ndarray:
    """The centring vector of a centred index (zeros otherwise), float32 [d]."""
    inf = fpp_index_get_info(h)
    c = np.zeros(inf["d"], dtype=np.float32)
    _check(lib().fpp_debug_center(h, c.ctypes.data_as(c_vp)))
    return c


def fpp_debug_set_partition_threshold(h, min_entries: int, range_bits: int = -1) -> None:
    """Queries with more probed entries than min_entries are deduplicated by id range, in ranges
    of 2^range_bits ids (< 0: the defaults)."""
    _check(lib().fpp_debug_set_partition_threshold(h, int(min_entries), int(range_bits)))


def fpp_debug_set_rerank_cut(h, enabled: bool) -> None:
    """Turn the BF16 rerank's cut (and the gather's matching threshold) off or on."""
    _check(lib().fpp_debug_set_rerank_cut(h, 1 if enabled else 0))


def fpp_normal_quantile(p: float) -> float:
    return float(lib().fpp_normal_quantile(float(p)))


def fpp_debug_build_records(h, t: int, device="cuda", stream=None):
    torch = _torch()
    inf = fpp_index_get_info(h)
    b = torch.empty((inf["n"], inf["iProbes"]), dtype=torch.int32, device=device)
    k = torch.empty((inf["n"], inf["iProbes"]), dtype=torch.float32, device=device)
    _check(lib().fpp_debug_build_records(h, t, c_vp(b.data_ptr()), c_vp(k.data_ptr()), _stream(stream)))
    return b, k


def fpp_debug_export_table(h, t: int):
    inf = fpp_index_get_info(h)
    sizes = fpp_index_table_sizes(h)
    off = np.zeros(inf["buckets_per_table"] + 1, dtype=np.uint32)
    ids = np.zeros(max(int(sizes[t]), 1), dtype=np.int32)
    _check(lib().fpp_debug_export_table(h, t, off.ctypes.data_as(c_vp), ids.ctypes.data_as(c_vp)))
    return off.astype(np.int64), ids[: int(sizes[t])]


def fpp_debug_probes(h, Q, qProbes: int, stream=None, probe_score: str = "sum"):
    torch = _torch()
    inf = fpp_index_get_info(h)
    pairs = inf["L"] * (inf["D"] if inf["l"] == 1 else inf["D"] ** 2)
    qc = min(qProbes, pairs)
    out = torch.empty((Q.shape[0], qc), dtype=torch.int64, device=Q.device)
    _check(lib().fpp_debug_probes(h, _dev(Q, torch.float32, "Q"), Q.shape[0], qProbes,
                                  PROBE_SCORES[probe_score], c_vp(out.data_ptr()), _stream(stream)))
    return out


def fpp_debug_export_store(h, store: str, stream=None):
    torch = _torch()
    inf = fpp_index_get_info(h)
    n, d = inf["n"], inf["d"]
    if store == "bf16":
        codes = torch.empty((n, d), dtype=torch.int16, device="cuda")
        scales = None
    elif store == "simhash":
        codes = torch.empty((n, (inf["simhash_bits"] + 31) // 32), dtype=torch.int32, device="cuda")
        scales = None
    else:
        codes = torch.empty((n, d), dtype=torch.uint8, device="cuda")
        scales = torch.empty(n, dtype=torch.float32, device="cuda")
    _check(lib().fpp_debug_export_store(h, STORES[store], c_vp(codes.data_ptr()),
                                        c_vp(scales.data_ptr()) if scales is not None else None,
                                        _stream(stream)))
    return codes, scales


# ------------------------------------------------------------------------------------------------
# serving
def fpp_server_create(h, *, scratch_bytes: int = 2 << 30, n_streams: int = 2, max_batch: int = 1024,
                      store: str = "fp32", rerank_R: int = 0, probe_score: str = "sum") -> c_vp:
    o = fpp_server_opts(scratch_bytes, n_streams, max_batch, STORES[store], rerank_R,
                        PROBE_SCORES[probe_score])
    sv = c_vp()
    _check(lib().fpp_server_create(h, ctypes.byref(o), ctypes.byref(sv)))
    return sv


def fpp_server_submit(sv, q_ptr: int, m: int, k: int, qProbes: int, ids_ptr: int, scores_ptr: int) -> int:
    """Submit m queries at device address q_ptr; results go to ids_ptr / scores_ptr ([m][k])."""
    t = c_i64()
    _check(lib().fpp_server_submit(sv, c_vp(q_ptr), m, k, qProbes, c_vp(ids_ptr), c_vp(scores_ptr),
                                   ctypes.byref(t)))
    return t.value


def fpp_server_replay(sv, q_ptr: int, t0_ns: int, arrive_ns, q_row, m, k, qProbes, ids_ptr: int,
                      scores_ptr: int, out_off):
    """Submit request i at CLOCK_MONOTONIC t0_ns + arrive_ns[i] (open-loop load generator in
    native code); returns the tickets. Host arrays: arrive_ns, q_row, out_off int64; m, k,
    qProbes int32; offsets count elements of the device buffers at q_ptr / ids_ptr / scores_ptr."""
    a = [np.ascontiguousarray(x, dtype=t) for x, t in ((arrive_ns, np.int64), (q_row, np.int64),
                                                         (m, np.int32), (k, np.int32),
                                                         (qProbes, np.int32), (out_off, np.int64))]
    n = a[0].shape[0]
    if any(x.shape != (n,) for x in a):
        raise ValueError("request arrays must have the same length")
    tickets = np.zeros(n, dtype=np.int64)
    ptr = lambda x: x.ctypes.data_as(c_vp)
    _check(lib().fpp_server_replay(sv, c_vp(q_ptr), n, t0_ns, ptr(a[0]), ptr(a[1]), ptr(a[2]), ptr(a[3]),
                                   ptr(a[4]), c_vp(ids_ptr), c_vp(scores_ptr), ptr(a[5]), ptr(tickets)))
    return tickets


def fpp_server_poll(sv, ticket: int):
    st, ts, td = c_i32(), c_i64(), c_i64()
    _check(lib().fpp_server_poll(sv, ticket, ctypes.byref(st), ctypes.byref(ts), ctypes.byref(td)))
    return st.value, ts.value, td.value


def fpp_server_wait(sv, ticket: int, timeout_ms: int = -1):
    st, ts, td = c_i32(), c_i64(), c_i64()
    _check(lib().fpp_server_wait(sv, ticket, timeout_ms, ctypes.byref(st), ctypes.byref(ts), ctypes.byref(td)))
    return st.value, ts.value, td.value


def fpp_server_get_stats(sv) -> dict:
    s = fpp_server_stats()
    _check(lib().fpp_server_get_stats(sv, ctypes.byref(s)))
    return {name: getattr(s, name) for name, _ in fpp_server_stats._fields_}


def fpp_server_debug_fail_batches(sv, n: int):
    """The next n batches fail after their first kernel (failure-handling tests)."""
    _check(lib().fpp_server_debug_fail_batches(sv, n))


def fpp_server_destroy(sv):
    if sv is not None and sv.value:
        lib().fpp_server_destroy(sv)
