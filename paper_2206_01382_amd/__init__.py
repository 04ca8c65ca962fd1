"""MI355X (gfx950) Falconn++ hot path: HIP kernels behind the C ABI of include/fpp.h.

The functions below are the C entry points with Python argument marshalling; see _lib.py.
``Index`` owns a handle and frees it when collected.
"""
from ._lib import (  # noqa: F401
    FPP_EINVAL, FPP_ECAPACITY, FPP_EHIP, FPP_ENOMEM, FPP_ESTATE, FPP_OK, FPP_STORE_BF16, FPP_STORE_FP32,
    FPP_STORE_FP8, FPP_FILTER_FRACTION, FPP_FILTER_THRESHOLD, FPP_PROBE_GAP, FPP_PROBE_SUM, FppError,
    LIB_PATH, fpp_build_index,
    fpp_debug_build_records, fpp_debug_center, fpp_debug_export_store, fpp_normal_quantile,
    fpp_debug_set_partition_threshold, fpp_debug_set_rerank_cut,
    fpp_debug_export_table, fpp_debug_probes, fpp_debug_query_lists, fpp_debug_signs, fpp_free_index,
    fpp_index_get_info, fpp_index_table_sizes, fpp_last_error, fpp_query, fpp_query_batch, fpp_query_ex_noalloc,
    fpp_query_workspace_bytes, fpp_server_create, fpp_server_debug_fail_batches, fpp_server_destroy,
    fpp_server_get_stats, fpp_server_poll,
    fpp_server_replay, fpp_server_submit, fpp_server_wait, fpp_version, lib,
)


class Index:
    """An index built on the GPU (Algorithm 1 over L tables); released with the object."""

    def __init__(self, X, L, D, alpha, iProbes, seed, **kw):
        self.handle = fpp_build_index(X, L, D, alpha, iProbes, seed, **kw)

    def query(self, Q, k, qProbes, **kw):
        return fpp_query(self.handle, Q, k, qProbes, **kw)

    def query_batch(self, Q, k, qProbes, **kw):
        return fpp_query_batch(self.handle, Q, k, qProbes, **kw)

    def info(self):
        return fpp_index_get_info(self.handle)

    def table_sizes(self):
        return fpp_index_table_sizes(self.handle)

    def close(self):
        if getattr(self, "handle", None) is not None:
            fpp_free_index(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
