"""MinHash / Min-Max LSH similarity search on MI355X (gfx950).

The hot path of the FAST earthquake-detection pipeline as scaled by Rong et
al. (VLDB 2018): signatures, band keys, hash-table buckets, the occurrence
filter, self-match exclusion and per-pair votes; the batched, bounded,
partitioned, query-only and serving forms of the search; the channel merge
and station-level diagonal clustering of its output; and fingerprint
extraction from waveforms; all in hand-written HIP kernels behind the C-ABI
of include/fast_lsh.h.  This package is the thin
Python binding over that library.
"""
from .fast_lsh import (CLUSTER_DTYPE, E_BUSY, E_CAPACITY, E_DEVICE, E_INVALID, E_NOMEM, KEEP_AUTO, MINHASH, MINMAX,
                       OK, QUEUE_OFF, FastLSH, FastLshError, Server, Stats, library, make_hash, n_funcs, plan_batch,
                       to_device_rows)

__all__ = ["CLUSTER_DTYPE", "E_BUSY", "E_CAPACITY", "E_DEVICE", "E_INVALID", "E_NOMEM", "KEEP_AUTO", "MINHASH",
           "MINMAX", "OK", "QUEUE_OFF",
           "FastLSH", "FastLshError", "Server", "Stats", "library", "make_hash", "n_funcs", "plan_batch",
           "to_device_rows"]
