"""CPU oracle — TEST INFRASTRUCTURE ONLY.

A plain, slow C implementation (``oracle.c``) of what the LSH similarity
search of Rong et al. (VLDB 2018) computes: MinHash / Min-Max signatures and
band keys (section 6.1, section 6.2, Appendix D Algorithm 1), hash tables,
the occurrence filter (section 6.5), self-match exclusion (section 7.1) and
per-pair vote counts (section 6.1 "Search", section 7.2 triplets).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the GPU path.
The readings taken where the paper is silent are listed in ``oracle.c``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_SRC = [os.path.join(_HERE, f) for f in ("oracle.c", "align.c", "partition.c")]

P = 2**31 - 1
MINHASH, MINMAX = 0, 1


def build() -> str:
    tmp = _SO + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-std=c11", *_SRC, "-o", tmp])
    os.replace(tmp, _SO)
    return _SO


class _Stats(ctypes.Structure):
    _fields_ = [(f, ctypes.c_uint64) for f in
                ("n_out", "e_raw", "e_voted", "n_distinct", "n_flagged", "max_bucket")]


_LIB = None
_LOCK = threading.Lock()
_vp, _u32, _u64 = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64


def _lib():
    global _LIB
    if _LIB is not None:
        return _LIB
    with _LOCK:
        if _LIB is not None:
            return _LIB
        if not os.path.exists(_SO):
            # Compiled only by build() (or __graft_entry__.build()), never
            # here: a process may already hold the GPU when it first calls in.
            raise RuntimeError(f"{_SO} is not built; run __graft_entry__.build() first")
        lib = ctypes.CDLL(_SO)
        lib.orc_splitmix64_stream.argtypes = [_u64, _u32, _vp]
        lib.orc_make_hash.argtypes = [_u64, _u32, _vp, _vp]
        lib.orc_hash.argtypes = [_u32, _u32, _u32]
        lib.orc_hash.restype = _u32
        lib.orc_key_bits.argtypes = [_u32]
        lib.orc_key_bits.restype = _u32
        lib.orc_band_key.argtypes = [_vp, _u32, _u32]
        lib.orc_band_key.restype = _u64
        lib.orc_band_keys.argtypes = [_u64, _vp, _u32, _u32, _vp]
        lib.orc_signatures.argtypes = [_u32, _u32, _u32, _u32, _vp, _vp, _u64, _vp, _u32, _vp, _vp, _vp]
        lib.orc_signatures.restype = ctypes.c_int
        lib.orc_search_keys.argtypes = [_u32, _u64, _vp, _u32, _u32, _u32, _u32, _u32,
                                        ctypes.POINTER(_vp), ctypes.POINTER(_vp), ctypes.POINTER(_vp),
                                        ctypes.POINTER(_Stats), _vp]
        lib.orc_search_keys.restype = ctypes.c_int
        lib.orc_table_scan.argtypes = [_u64, _vp, _u32, _u32, _vp, ctypes.POINTER(_u64), ctypes.POINTER(_u64),
                                       _u32, _u32, _vp, ctypes.POINTER(_vp), ctypes.POINTER(_u64)]
        lib.orc_table_scan.restype = ctypes.c_int
        lib.orc_count_votes.argtypes = [_vp, _u64, _vp, _u32, ctypes.POINTER(_vp), ctypes.POINTER(_vp),
                                        ctypes.POINTER(_vp), ctypes.POINTER(_Stats)]
        lib.orc_count_votes.restype = ctypes.c_int
        lib.orc_pair_votes.argtypes = [_u32, _u64, _vp, _u64, _u64]
        lib.orc_pair_votes.restype = _u32
        lib.orc_free.argtypes = [_vp]
        lib.orc_channel_merge.argtypes = [_u32, _vp, _vp, _vp, _vp, _u32, ctypes.POINTER(_vp), ctypes.POINTER(_vp),
                                          ctypes.POINTER(_vp), ctypes.POINTER(_u64)]
        lib.orc_channel_merge.restype = ctypes.c_int
        lib.orc_station_clusters.argtypes = [_u64, _vp, _vp, _vp, _u32, _u32, _u32, _u64, ctypes.POINTER(_vp),
                                             ctypes.POINTER(_u64)]
        lib.orc_station_clusters.restype = ctypes.c_int
        lib.orc_query_keys.argtypes = [_u32, _u64, _vp, _u64, _vp, _u32, ctypes.POINTER(_vp), ctypes.POINTER(_vp),
                                       ctypes.POINTER(_vp), ctypes.POINTER(_u64), ctypes.POINTER(_u64)]
        lib.orc_query_keys.restype = ctypes.c_int
        lib.orc_search_partitioned_keys.argtypes = [_u32, _u64, _vp, _u32, _u32, _u32, _u32, _u32,
                                                    ctypes.POINTER(_vp), ctypes.POINTER(_vp), ctypes.POINTER(_vp),
                                                    ctypes.POINTER(_Stats), _vp]
        lib.orc_search_partitioned_keys.restype = ctypes.c_int
        lib.orc_max_threads.restype = ctypes.c_int
        lib.orc_set_threads.argtypes = [ctypes.c_int]
        _LIB = lib
    return _LIB


@dataclass
class Stats:
    n_out: int
    e_raw: int
    e_voted: int
    n_distinct: int
    n_flagged: int
    max_bucket: int


def splitmix64_stream(seed: int, count: int) -> np.ndarray:
    out = np.empty(count, dtype=np.uint64)
    _lib().orc_splitmix64_stream(seed, count, out.ctypes.data)
    return out


def n_funcs(t: int, r: int, scheme: int) -> int:
    return t * r if scheme == MINHASH else t * (r // 2)


def make_hash(seed: int, nf: int):
    a = np.empty(nf, dtype=np.uint32)
    b = np.empty(nf, dtype=np.uint32)
    _lib().orc_make_hash(seed, nf, a.ctypes.data, b.ctypes.data)
    return a, b


def hash_value(a: int, b: int, x: int) -> int:
    return int(_lib().orc_hash(a, b, x))


def key_bits(dim: int) -> int:
    return int(_lib().orc_key_bits(dim))


def band_key(argx, dim: int) -> int:
    arr = np.ascontiguousarray(argx, dtype=np.uint32)
    return int(_lib().orc_band_key(arr.ctypes.data, len(arr), dim))


def band_keys(argx, dim: int) -> np.ndarray:
    """band_key of every row of a uint32[n, r] array of attaining indices."""
    arr = np.ascontiguousarray(argx, dtype=np.uint32)
    n, r = arr.shape
    out = np.empty(n, dtype=np.uint64)
    _lib().orc_band_keys(n, arr.ctypes.data, r, dim, out.ctypes.data)
    return out


def _rows(rows):
    """Accept a uint16[n, nnz] array (fixed nnz) or a (indices, offsets) pair."""
    if isinstance(rows, tuple):
        ind, off = rows
        ind = np.ascontiguousarray(ind, dtype=np.uint16)
        off = np.ascontiguousarray(off, dtype=np.uint64)
        return ind, off, len(off) - 1, 0
    rows = np.ascontiguousarray(rows, dtype=np.uint16)
    return rows, None, rows.shape[0], rows.shape[1]


def signatures(rows, dim: int, t: int, r: int, scheme: int, a, b, with_values: bool = False):
    """keys uint64[t, n]; with ``with_values`` also the values uint32[n, t, r]."""
    ind, off, n, nnz = _rows(rows)
    a = np.ascontiguousarray(a, dtype=np.uint32)
    b = np.ascontiguousarray(b, dtype=np.uint32)
    keys = np.empty((t, n), dtype=np.uint64)
    sigs = np.empty((n, t, r), dtype=np.uint32) if with_values else None
    rc = _lib().orc_signatures(dim, t, r, scheme, a.ctypes.data, b.ctypes.data, n,
                               off.ctypes.data if off is not None else None, nnz, ind.ctypes.data,
                               keys.ctypes.data, sigs.ctypes.data if with_values else None)
    if rc != 0:
        raise ValueError("oracle: invalid hash parameters or fingerprints")
    return (keys, sigs) if with_values else keys


def _take_triplets(pi, pj, pv, m):
    cast = lambda p, ct: np.ctypeslib.as_array(ctypes.cast(p, ctypes.POINTER(ct)), (m,)).copy()
    oi = cast(pi, ctypes.c_uint32) if m else np.empty(0, np.uint32)
    oj = cast(pj, ctypes.c_uint32) if m else np.empty(0, np.uint32)
    ov = cast(pv, ctypes.c_uint8) if m else np.empty(0, np.uint8)
    for p in (pi, pj, pv):
        _lib().orc_free(p)
    return oi, oj, ov


def search_keys(keys: np.ndarray, min_lag: int, min_votes: int, occ_num: int = 0, occ_den: int = 0,
                want_flags: bool = False, parts: int = 1):
    """(i, j, votes, Stats[, flags]) from table-major band keys uint64[t, n];
    ``parts`` vote partitions (ranges of i) are counted one after another."""
    keys = np.ascontiguousarray(keys, dtype=np.uint64)
    t, n = keys.shape
    pi, pj, pv = _vp(), _vp(), _vp()
    st = _Stats()
    flags = np.empty(n, dtype=np.uint8) if want_flags else None
    rc = _lib().orc_search_keys(t, n, keys.ctypes.data, min_lag, min_votes, occ_num, occ_den, parts,
                                ctypes.byref(pi), ctypes.byref(pj), ctypes.byref(pv), ctypes.byref(st),
                                flags.ctypes.data if want_flags else None)
    if rc == 2:
        raise MemoryError("oracle: out of host memory")
    if rc != 0:
        raise ValueError("oracle: invalid search parameters")
    oi, oj, ov = _take_triplets(pi, pj, pv, st.n_out)
    stats = Stats(*[int(getattr(st, f)) for f, _ in _Stats._fields_])
    return (oi, oj, ov, stats, flags) if want_flags else (oi, oj, ov, stats)


class TableScan:
    """A search taken one table at a time (keys of one table in memory at
    once): ``add_table`` sorts a table, accumulates its bucket counters and
    exclusions and collects its candidate pairs whose i lies in ``ranges``;
    ``result`` counts the votes of the collected pairs."""

    def __init__(self, n: int, occ_num: int, occ_den: int, min_lag: int, ranges):
        self.n, self.occ_num, self.occ_den, self.min_lag = n, occ_num, occ_den, min_lag
        self.ranges = np.ascontiguousarray(np.asarray(ranges, dtype=np.uint64).reshape(-1))
        self.flags = np.zeros(max(n, 1), dtype=np.uint8)
        self.e_raw = _u64(0)
        self.max_bucket = _u64(0)
        self._pairs = _vp()
        self._cnt = _u64(0)
        self.tables = 0

    def add_table(self, keys_u: np.ndarray):
        keys_u = np.ascontiguousarray(keys_u, dtype=np.uint64)
        assert keys_u.shape == (self.n,)
        rc = _lib().orc_table_scan(self.n, keys_u.ctypes.data, self.occ_num, self.occ_den, self.flags.ctypes.data,
                                   ctypes.byref(self.e_raw), ctypes.byref(self.max_bucket), self.min_lag,
                                   len(self.ranges) // 2, self.ranges.ctypes.data, ctypes.byref(self._pairs),
                                   ctypes.byref(self._cnt))
        if rc != 0:
            raise MemoryError("oracle: out of host memory")
        self.tables += 1

    @property
    def pairs_collected(self) -> int:
        return int(self._cnt.value)

    def result(self, min_votes: int):
        """(i, j, votes, Stats) of the collected ranges; e_raw, max_bucket and
        n_flagged are those of the whole search."""
        pi, pj, pv = _vp(), _vp(), _vp()
        st = _Stats()
        rc = _lib().orc_count_votes(self._pairs, self._cnt.value, self.flags.ctypes.data, min_votes,
                                    ctypes.byref(pi), ctypes.byref(pj), ctypes.byref(pv), ctypes.byref(st))
        if rc != 0:
            raise MemoryError("oracle: out of host memory")
        oi, oj, ov = _take_triplets(pi, pj, pv, st.n_out)
        stats = Stats(n_out=int(st.n_out), e_raw=int(self.e_raw.value), e_voted=int(st.e_voted),
                      n_distinct=int(st.n_distinct), n_flagged=int(self.flags[:self.n].sum()),
                      max_bucket=int(self.max_bucket.value))
        return oi, oj, ov, stats

    def close(self):
        if self._pairs:
            _lib().orc_free(self._pairs)
            self._pairs = _vp()
            self._cnt = _u64(0)

    def __del__(self):
        self.close()


def search(rows, dim: int, t: int, r: int, scheme: int, a, b, min_lag: int, min_votes: int,
           occ_num: int = 0, occ_den: int = 0):
    keys = signatures(rows, dim, t, r, scheme, a, b)
    return search_keys(keys, min_lag, min_votes, occ_num, occ_den)


def max_threads() -> int:
    return int(_lib().orc_max_threads())


def set_threads(n: int) -> None:
    """Threads of later oracle calls (timing only; results do not change)."""
    _lib().orc_set_threads(int(n))


def pair_votes(keys: np.ndarray, i: int, j: int) -> int:
    keys = np.ascontiguousarray(keys, dtype=np.uint64)
    t, n = keys.shape
    return int(_lib().orc_pair_votes(t, n, keys.ctypes.data, i, j))


# --------------------------------------------------------------------------
# Spatiotemporal alignment (section 7): channel merge and station clusters
# --------------------------------------------------------------------------
CLUSTER_DTYPE = np.dtype([("dt_min", "<u4"), ("dt_max", "<u4"), ("idx1_min", "<u4"), ("idx1_max", "<u4"),
                          ("n_entries", "<u4"), ("peak_sim", "<u4"), ("peak_dt", "<u4"), ("peak_idx1", "<u4"),
                          ("sim_sum", "<u8")])


def channel_merge(channels, min_sim: int):
    """Channel-level sort-merge-reduce of search outputs [(i, j, votes), ...]
    of one station's channels: (dt, idx1, sim) uint32 arrays ordered by
    (dt, idx1), sums of sim >= min_sim only."""
    arrs = [(np.ascontiguousarray(i, dtype=np.uint32), np.ascontiguousarray(j, dtype=np.uint32),
             np.ascontiguousarray(v, dtype=np.uint8)) for i, j, v in channels]
    n = len(arrs)
    counts = np.array([len(a[0]) for a in arrs] or [0], dtype=np.uint64)
    ptr = lambda q: np.array([a[q].ctypes.data for a in arrs] or [0], dtype=np.uint64)
    pi, pj, pv = ptr(0), ptr(1), ptr(2)
    odt, oid, osm, m = _vp(), _vp(), _vp(), _u64()
    rc = _lib().orc_channel_merge(n, counts.ctypes.data, pi.ctypes.data, pj.ctypes.data, pv.ctypes.data, min_sim,
                                  ctypes.byref(odt), ctypes.byref(oid), ctypes.byref(osm), ctypes.byref(m))
    if rc == 1:
        raise ValueError("oracle: a pair with j <= i")
    if rc != 0:
        raise MemoryError("oracle: out of host memory")
    k = int(m.value)
    out = []
    for p in (odt, oid, osm):
        a = np.ctypeslib.as_array(ctypes.cast(p, ctypes.POINTER(ctypes.c_uint32)), (k,)).copy() if k else \
            np.empty(0, np.uint32)
        _lib().orc_free(p)
        out.append(a)
    return tuple(out)


def station_clusters(dt, idx1, sim, max_gap: int, max_width: int, min_entries: int = 1, min_sum: int = 0):
    """Station-level diagonal clusters of (dt, idx1)-ordered entries: a
    structured array (CLUSTER_DTYPE) in the order of each cluster's first entry."""
    dt = np.ascontiguousarray(dt, dtype=np.uint32)
    idx1 = np.ascontiguousarray(idx1, dtype=np.uint32)
    sim = np.ascontiguousarray(sim, dtype=np.uint32)
    p, m = _vp(), _u64()
    rc = _lib().orc_station_clusters(len(dt), dt.ctypes.data, idx1.ctypes.data, sim.ctypes.data, max_gap, max_width,
                                     min_entries, min_sum, ctypes.byref(p), ctypes.byref(m))
    if rc == 1:
        raise ValueError("oracle: entries not strictly ordered by (dt, idx1)")
    if rc != 0:
        raise MemoryError("oracle: out of host memory")
    k = int(m.value)
    out = np.empty(k, dtype=CLUSTER_DTYPE)
    if k:
        ctypes.memmove(out.ctypes.data, p, k * CLUSTER_DTYPE.itemsize)
    _lib().orc_free(p)
    return out


# --------------------------------------------------------------------------
# Section 6.4 / 6.5 forms: query-only hashing, partitioned search with the
# dynamic occurrence filter
# --------------------------------------------------------------------------
def query_keys(qkeys: np.ndarray, dkeys: np.ndarray, min_votes: int):
    """(q, x, votes, n_matches): query-only hashing from band keys uint64[t, nq]
    and uint64[t, nd]; pairs with at least min_votes votes, ordered by (q, x)."""
    qkeys = np.ascontiguousarray(qkeys, dtype=np.uint64)
    dkeys = np.ascontiguousarray(dkeys, dtype=np.uint64)
    t, nq = qkeys.shape
    t2, nd = dkeys.shape
    assert t == t2
    pq, px, pv, m, nc = _vp(), _vp(), _vp(), _u64(), _u64()
    rc = _lib().orc_query_keys(t, nq, qkeys.ctypes.data, nd, dkeys.ctypes.data, min_votes, ctypes.byref(pq),
                               ctypes.byref(px), ctypes.byref(pv), ctypes.byref(m), ctypes.byref(nc))
    if rc == 1:
        raise ValueError("oracle: invalid query arguments")
    if rc != 0:
        raise MemoryError("oracle: out of host memory")
    q, x, v = _take_triplets(pq, px, pv, int(m.value))
    return q, x, v, int(nc.value)


def query(queries, dataset, dim: int, t: int, r: int, scheme: int, a, b, min_votes: int):
    """Query-only hashing from fingerprints (signatures, then query_keys)."""
    return query_keys(signatures(queries, dim, t, r, scheme, a, b), signatures(dataset, dim, t, r, scheme, a, b),
                      min_votes)


def search_partitioned_keys(keys: np.ndarray, min_lag: int, min_votes: int, occ_num: int, occ_den: int,
                            n_parts: int, want_excluded: bool = False):
    """(i, j, votes, Stats[, excluded]): partitioned search with the dynamic
    occurrence filter from band keys uint64[t, n]."""
    keys = np.ascontiguousarray(keys, dtype=np.uint64)
    t, n = keys.shape
    pi, pj, pv = _vp(), _vp(), _vp()
    st = _Stats()
    ex = np.empty(max(n, 1), dtype=np.uint8)
    rc = _lib().orc_search_partitioned_keys(t, n, keys.ctypes.data, min_lag, min_votes, occ_num, occ_den, n_parts,
                                            ctypes.byref(pi), ctypes.byref(pj), ctypes.byref(pv), ctypes.byref(st),
                                            ex.ctypes.data)
    if rc == 1:
        raise ValueError("oracle: invalid partitioned-search arguments")
    if rc != 0:
        raise MemoryError("oracle: out of host memory")
    oi, oj, ov = _take_triplets(pi, pj, pv, st.n_out)
    stats = Stats(*[int(getattr(st, f)) for f, _ in _Stats._fields_])
    return (oi, oj, ov, stats, ex[:n]) if want_excluded else (oi, oj, ov, stats)
