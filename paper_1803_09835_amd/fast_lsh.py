"""Python binding of the fast_lsh C-ABI (include/fast_lsh.h).

Argument marshalling only: every step of the search runs in the HIP library
``libfast_lsh.so``.  PyTorch supplies device memory and the stream.  There is
no fallback: without the built library every call raises.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfast_lsh.so")

OK, E_INVALID, E_NOMEM, E_CAPACITY, E_DEVICE, E_BUSY = range(6)
MINHASH, MINMAX = 0, 1
WANT_DISTINCT, USE_GRAPH = 1, 2
MAX_STATIONS = 16

_vp, _u32, _u64, _i32 = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int


class Hash(ctypes.Structure):
    _fields_ = [("dim", _u32), ("num_tables", _u32), ("band_rows", _u32), ("scheme", _u32),
                ("a", _vp), ("b", _vp)]


class Fps(ctypes.Structure):
    _fields_ = [("indices", _vp), ("offsets", _vp), ("fixed_nnz", _u32), ("reserved", _u32), ("n", _u64)]


class Filter(ctypes.Structure):
    _fields_ = [("min_lag", _u32), ("min_votes", _u32), ("occ_num", _u32), ("occ_den", _u32)]


class _Stats(ctypes.Structure):
    _fields_ = [(f, _u64) for f in ("n_out", "e_raw", "e_voted", "n_distinct", "n_flagged", "max_bucket")]


PROFILE_STAGES = ("signatures", "group", "buckets", "big_bins", "pairs", "big_pairs", "output", "graph", "split_keys",
                  "channel_merge", "clusters", "fingerprints", "spectrogram", "pair_checks")


class Config(ctypes.Structure):
    _fields_ = [("radix_tile", _u32), ("bucket_chunk", _u32), ("autotune", _u32), ("bin_bits", _u32),
                ("keep_groups", _u32), ("queue_slot", _u32)]


KEEP_AUTO = 0xFFFFFFFF
QUEUE_OFF = 0xFFFFFFFF


class _Profile(ctypes.Structure):
    _fields_ = [("ms", ctypes.c_double * len(PROFILE_STAGES)), ("launches", ctypes.c_uint64 * len(PROFILE_STAGES))]


class Pairs(ctypes.Structure):
    _fields_ = [("i", _vp), ("j", _vp), ("votes", _vp), ("count", _u64)]


class ClusterParams(ctypes.Structure):
    _fields_ = [("max_gap", _u32), ("max_width", _u32), ("min_entries", _u32), ("reserved", _u32),
                ("min_sum", _u64)]


# fast_lsh_cluster as a numpy record (40 bytes)
CLUSTER_DTYPE = np.dtype([("dt_min", "<u4"), ("dt_max", "<u4"), ("idx1_min", "<u4"), ("idx1_max", "<u4"),
                          ("n_entries", "<u4"), ("peak_sim", "<u4"), ("peak_dt", "<u4"), ("peak_idx1", "<u4"),
                          ("sim_sum", "<u8")])


class FpParams(ctypes.Structure):
    _fields_ = [(f, _u32) for f in ("window", "hop", "band_lo", "band_hi", "fp_frames", "time_ds", "fp_lag", "top_k")]


class _Work(ctypes.Structure):
    _fields_ = [(f, ctypes.c_uint64) for f in ("big_voted", "big_members", "big_candidates", "search_calls",
                                               "pair_redos")]


@dataclass
class Stats:
    n_out: int
    e_raw: int
    e_voted: int
    n_distinct: int
    n_flagged: int
    max_bucket: int


class FastLshError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"fast_lsh error {code}: {msg}")
        self.code = code


_LIB = None


def library():
    """Load libfast_lsh.so (raises if it has not been built)."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise FastLshError(E_DEVICE, f"HIP library missing: {LIB_PATH} (run __graft_entry__.build())")
        lib = ctypes.CDLL(LIB_PATH)
        lib.fast_lsh_version.restype = _i32
        lib.fast_lsh_last_error.restype = ctypes.c_char_p
        lib.fast_lsh_ctx_create.argtypes = [_i32, _vp, _u64, ctypes.POINTER(_vp)]
        lib.fast_lsh_ctx_destroy.argtypes = [_vp]
        lib.fast_lsh_make_hash.argtypes = [_u64, _u32, _vp, _vp]
        lib.fast_lsh_signatures.argtypes = [_vp, ctypes.POINTER(Hash), ctypes.POINTER(Fps), _u32, _u32, _vp, _vp]
        lib.fast_lsh_search.argtypes = [_vp, ctypes.POINTER(Hash), ctypes.POINTER(Fps), ctypes.POINTER(Filter),
                                        _vp, _vp, _vp, _u64, ctypes.POINTER(_Stats)]
        lib.fast_lsh_search_ex.argtypes = [_vp, ctypes.POINTER(Hash), ctypes.POINTER(Fps), ctypes.POINTER(Filter),
                                           _u32, _vp, _vp, _vp, _u64, ctypes.POINTER(_Stats)]
        lib.fast_lsh_search_batched.argtypes = [_vp, ctypes.POINTER(Hash), _u32, ctypes.POINTER(Fps),
                                                ctypes.POINTER(Filter), _u32, _vp, _vp, _vp, _u64,
                                                ctypes.POINTER(_u64), ctypes.POINTER(_Stats)]
        lib.fast_lsh_search_bounded.argtypes = [_vp, ctypes.POINTER(Hash), ctypes.POINTER(Fps),
                                                ctypes.POINTER(Filter), _u32, _u32, _vp, _vp, _vp, _u64,
                                                ctypes.POINTER(_Stats)]
        lib.fast_lsh_copy_result.argtypes = [_vp, _vp, _vp, _vp, _u64]
        lib.fast_lsh_configure.argtypes = [_vp, ctypes.POINTER(Config)]
        lib.fast_lsh_config_used.argtypes = [_vp, ctypes.POINTER(Config)]
        lib.fast_lsh_workspace_bytes.argtypes = [_vp, ctypes.POINTER(_u64)]
        lib.fast_lsh_profile_enable.argtypes = [_vp, _i32]
        lib.fast_lsh_profile_read.argtypes = [_vp, ctypes.POINTER(_Profile)]
        lib.fast_lsh_last_work.argtypes = [_vp, ctypes.POINTER(_Work)]
        lib.fast_lsh_channel_merge.argtypes = [_vp, _u32, ctypes.POINTER(Pairs), _u64, _u32, _vp, _vp, _vp, _u64,
                                               ctypes.POINTER(_u64)]
        lib.fast_lsh_channel_merge_noalloc.argtypes = lib.fast_lsh_channel_merge.argtypes
        lib.fast_lsh_search_partitioned.argtypes = [_vp, ctypes.POINTER(Hash), ctypes.POINTER(Fps),
                                                    ctypes.POINTER(Filter), _u32, _u32, _vp, _vp, _vp, _u64,
                                                    ctypes.POINTER(_Stats)]
        lib.fast_lsh_fingerprints.argtypes = [_vp, _vp, _u64, ctypes.POINTER(FpParams), _vp, _u64, _vp, _vp, _u64,
                                              ctypes.POINTER(_u64), _vp]
        lib.fast_lsh_query.argtypes = [_vp, ctypes.POINTER(Hash), ctypes.POINTER(Fps), ctypes.POINTER(Fps), _u32,
                                       _vp, _vp, _vp, _u64, ctypes.POINTER(_Stats)]
        lib.fast_lsh_station_clusters.argtypes = [_vp, _vp, _vp, _vp, _u64, ctypes.POINTER(ClusterParams), _vp,
                                                  _u64, ctypes.POINTER(_u64)]
        _LIB = lib
    return _LIB


def _check(rc: int):
    if rc != OK:
        raise FastLshError(rc, library().fast_lsh_last_error().decode())


def n_funcs(t: int, r: int, scheme: int) -> int:
    return t * r if scheme == MINHASH else t * (r // 2)


def make_hash(seed: int, nf: int):
    """(a, b) uint32 arrays of the seeded hash family (host-side)."""
    a = np.empty(nf, np.uint32)
    b = np.empty(nf, np.uint32)
    _check(library().fast_lsh_make_hash(seed, nf, a.ctypes.data, b.ctypes.data))
    return a, b


def _hash_struct(dim, t, r, scheme, a, b):
    a = np.ascontiguousarray(a, np.uint32)
    b = np.ascontiguousarray(b, np.uint32)
    h = Hash(dim, t, r, scheme, a.ctypes.data, b.ctypes.data)
    return h, (a, b)


def _fps_struct(rows):
    """rows: a CUDA tensor [n, nnz] of 16-bit indices, or (indices, offsets)
    CUDA tensors (16-bit indices, 64-bit offsets with n+1 entries)."""
    if isinstance(rows, tuple):
        ind, off = rows
        assert ind.is_cuda and off.is_cuda and ind.element_size() == 2 and off.element_size() == 8
        n = off.numel() - 1
        return Fps(ind.data_ptr(), off.data_ptr(), 0, 0, n), (ind, off)
    assert rows.is_cuda and rows.element_size() == 2 and rows.dim() == 2 and rows.is_contiguous()
    return Fps(rows.data_ptr(), None, rows.shape[1], 0, rows.shape[0]), (rows,)


def to_device_rows(rows_np: np.ndarray, device="cuda") -> torch.Tensor:
    """uint16 numpy rows -> int16 CUDA tensor with the same bits."""
    return torch.from_numpy(np.ascontiguousarray(rows_np).view(np.int16)).to(device)


class FastLSH:
    """One library context on a device, ordered on a torch stream."""

    def __init__(self, device: int = 0, stream: torch.cuda.Stream | None = None, hbm_budget: int = 0):
        self.device = device
        self.stream = stream if stream is not None else torch.cuda.current_stream(device)
        ctx = _vp()
        _check(library().fast_lsh_ctx_create(device, self.stream.cuda_stream, hbm_budget, ctypes.byref(ctx)))
        self._ctx = ctx

    def close(self):
        if getattr(self, "_ctx", None):
            library().fast_lsh_ctx_destroy(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def workspace_bytes(self) -> int:
        """Device memory the context's workspace holds now."""
        v = _u64()
        _check(library().fast_lsh_workspace_bytes(self._ctx, ctypes.byref(v)))
        return int(v.value)

    def profile_enable(self, on: bool = True):
        """Start (and reset) per-stage kernel timing with HIP events on the context stream."""
        _check(library().fast_lsh_profile_enable(self._ctx, 1 if on else 0))

    def profile_read(self) -> dict:
        """{stage: (summed kernel ms, timed launches)} since profile_enable."""
        p = _Profile()
        _check(library().fast_lsh_profile_read(self._ctx, ctypes.byref(p)))
        return {name: (p.ms[k], int(p.launches[k])) for k, name in enumerate(PROFILE_STAGES)}

    def search_partitioned(self, rows, dim, t, r, scheme, a, b, min_lag, min_votes, occ_num=0, occ_den=0,
                           n_partitions=1, want_distinct=False, capacity: int | None = None):
        """Partitioned search with the dynamic occurrence filter (sections 6.4,
        6.5): sorted (i, j, votes) CUDA tensors and Stats."""
        h, keep = _hash_struct(dim, t, r, scheme, a, b)
        f, keep2 = _fps_struct(rows)
        flt = Filter(min_lag, min_votes, occ_num, occ_den)
        flags = WANT_DISTINCT if want_distinct else 0
        cap = max(1, f.n // 4) if capacity is None else capacity
        oi, oj, ov = self._outputs(cap)
        st = _Stats()
        rc = library().fast_lsh_search_partitioned(self._ctx, ctypes.byref(h), ctypes.byref(f), ctypes.byref(flt),
                                                   flags, n_partitions, oi.data_ptr(), oj.data_ptr(), ov.data_ptr(),
                                                   cap, ctypes.byref(st))
        if rc == E_CAPACITY and capacity is None:
            rc, (oi, oj, ov) = self._refetch(rc, st.n_out, capacity)
        _check(rc)
        m = st.n_out
        return oi[:m], oj[:m], ov[:m], Stats(*[int(getattr(st, k)) for k, _ in _Stats._fields_])

    def fingerprints(self, samples, sample_ids, window=200, hop=10, band_lo=4, band_hi=36, fp_frames=128, time_ds=2,
                     fp_lag=10, top_k=200, want_stats=False):
        """Fingerprints (section 5) of a float32 CUDA tensor of samples: an
        int16 CUDA tensor [n_fp, top_k] of bit indices (uint16 bits), the
        per-fingerprint counts, and (want_stats) the medians and MADs."""
        prm = FpParams(window, hop, band_lo, band_hi, fp_frames, time_ds, fp_lag, top_k)
        assert samples.is_cuda and samples.dtype == torch.float32 and samples.is_contiguous()
        ids = torch.as_tensor(sample_ids, dtype=torch.int64, device=f"cuda:{self.device}").contiguous()
        nfp = _u64()
        rc = library().fast_lsh_fingerprints(self._ctx, samples.data_ptr(), samples.numel(), ctypes.byref(prm),
                                             ids.data_ptr(), ids.numel(), None, None, 0, ctypes.byref(nfp), None)
        if rc not in (OK, E_CAPACITY):
            _check(rc)
        n = int(nfp.value)
        dev = f"cuda:{self.device}"
        out = torch.empty((max(n, 1), top_k), dtype=torch.int16, device=dev)
        cnt = torch.empty(max(n, 1), dtype=torch.int32, device=dev)
        nc = (band_hi - band_lo) * (fp_frames // time_ds)
        stats = torch.empty(2 * nc, dtype=torch.float32, device=dev) if want_stats else None
        _check(library().fast_lsh_fingerprints(self._ctx, samples.data_ptr(), samples.numel(), ctypes.byref(prm),
                                               ids.data_ptr(), ids.numel(), out.data_ptr(), cnt.data_ptr(), n,
                                               ctypes.byref(nfp), stats.data_ptr() if want_stats else None))
        res = (out[:n], cnt[:n])
        return res + ((stats[:nc], stats[nc:]),) if want_stats else res

    def query(self, queries, dataset, dim, t, r, scheme, a, b, min_votes, capacity: int | None = None):
        """Query-only hashing (section 6.4): (q, x, votes) CUDA tensors of the
        (query, item) pairs with at least min_votes votes, and Stats."""
        h, keep = _hash_struct(dim, t, r, scheme, a, b)
        fq, kq = _fps_struct(queries)
        fd, kd = _fps_struct(dataset)
        cap = max(1, 4 * fq.n) if capacity is None else capacity
        st = _Stats()
        while True:
            oq, ox, ov = self._outputs(cap)
            rc = library().fast_lsh_query(self._ctx, ctypes.byref(h), ctypes.byref(fq), ctypes.byref(fd), min_votes,
                                          oq.data_ptr(), ox.data_ptr(), ov.data_ptr(), cap, ctypes.byref(st))
            if rc == E_CAPACITY and capacity is None:
                cap = st.n_out
                continue
            break
        _check(rc)
        m = st.n_out
        return oq[:m], ox[:m], ov[:m], Stats(*[int(getattr(st, k)) for k, _ in _Stats._fields_])

    def channel_merge(self, channels, n_fingerprints: int, min_sim: int, capacity: int | None = None,
                      noalloc: bool = False):
        """Combined similarity of one station's channels (section 7.2): channels
        is a list of (i, j, votes) CUDA tensors (search outputs); returns
        (dt, idx1, sim) int32 CUDA tensors ordered by (dt, idx1).  noalloc:
        the library call that allocates no device memory (fixed scratch)."""
        keep = [(i.contiguous(), j.contiguous(), v.contiguous()) for i, j, v in channels]
        arr = (Pairs * max(1, len(keep)))()
        for q, (i, j, v) in enumerate(keep):
            assert i.is_cuda and i.element_size() == 4 and j.element_size() == 4 and v.element_size() == 1
            arr[q] = Pairs(i.data_ptr(), j.data_ptr(), v.data_ptr(), i.numel())
        total = sum(i.numel() for i, _, _ in keep)
        cap = max(1, total) if capacity is None else capacity
        out = [torch.empty(max(cap, 1), dtype=torch.int32, device=f"cuda:{self.device}") for _ in range(3)]
        m = _u64()
        fn = library().fast_lsh_channel_merge_noalloc if noalloc else library().fast_lsh_channel_merge
        rc = fn(self._ctx, len(keep), arr, n_fingerprints, min_sim, out[0].data_ptr(), out[1].data_ptr(),
                out[2].data_ptr(), cap, ctypes.byref(m))
        _check(rc)
        k = int(m.value)
        return out[0][:k], out[1][:k], out[2][:k]

    def station_clusters(self, dt, idx1, sim, max_gap: int, max_width: int, min_entries: int = 1, min_sum: int = 0,
                         capacity: int | None = None):
        """Diagonal clusters of (dt, idx1)-ordered entries (section 7.2): a
        uint8 CUDA tensor of CLUSTER_DTYPE records ([k, 40] bytes)."""
        dt, idx1, sim = dt.contiguous(), idx1.contiguous(), sim.contiguous()
        n = dt.numel()
        assert idx1.numel() == n and sim.numel() == n
        assert all(x.is_cuda and x.element_size() == 4 for x in (dt, idx1, sim))
        cap = max(1, n) if capacity is None else capacity
        out = torch.empty((max(cap, 1), CLUSTER_DTYPE.itemsize), dtype=torch.uint8, device=f"cuda:{self.device}")
        prm = ClusterParams(max_gap, max_width, min_entries, 0, min_sum)
        m = _u64()
        _check(library().fast_lsh_station_clusters(self._ctx, dt.data_ptr(), idx1.data_ptr(), sim.data_ptr(), n,
                                                   ctypes.byref(prm), out.data_ptr(), cap, ctypes.byref(m)))
        return out[: int(m.value)]

    def last_work(self) -> dict:
        """Work counters of the last search (tiled buckets: voted pairs,
        members, in-bucket pairs; searches completed)."""
        w = _Work()
        _check(library().fast_lsh_last_work(self._ctx, ctypes.byref(w)))
        return {f: int(getattr(w, f)) for f, _ in _Work._fields_}

    def configure(self, radix_tile: int = 0, bucket_chunk: int = 0, autotune: bool = False, bin_bits: int = 0,
                  keep_groups: int = KEEP_AUTO, queue_slot: int = 0):
        """Launch shapes of later searches (0 keeps the current tile and chunk;
        bin_bits 0 is the automatic rule; keep_groups caps the table groups
        the bounded search keeps between its passes, KEEP_AUTO: as many as
        HBM holds; queue_slot: candidate queue entries per spread slot, 0
        automatic, QUEUE_OFF checks in place)."""
        _check(library().fast_lsh_configure(self._ctx, ctypes.byref(Config(radix_tile, bucket_chunk,
                                                                            1 if autotune else 0, bin_bits,
                                                                            keep_groups, queue_slot))))

    def config_used(self) -> dict:
        """Launch shapes of the last search (the tuner's choice when autotuning)."""
        c = Config()
        _check(library().fast_lsh_config_used(self._ctx, ctypes.byref(c)))
        return {"radix_tile": c.radix_tile, "bucket_chunk": c.bucket_chunk, "autotune": bool(c.autotune),
                "bin_bits": c.bin_bits, "keep_groups": c.keep_groups, "queue_slot": c.queue_slot}

    def signatures(self, rows, dim, t, r, scheme, a, b, table_begin=0, table_count=None, with_values=False):
        """Band keys as int64 [table_count, n] (uint64 bit pattern); with
        ``with_values`` also the hash values int32 [n, table_count, r]."""
        tc = t - table_begin if table_count is None else table_count
        h, keep = _hash_struct(dim, t, r, scheme, a, b)
        f, keep2 = _fps_struct(rows)
        dev = torch.device("cuda", self.device)
        keys = torch.empty((tc, f.n), dtype=torch.int64, device=dev)
        sigs = torch.empty((f.n, tc, r), dtype=torch.int32, device=dev) if with_values else None
        _check(library().fast_lsh_signatures(self._ctx, ctypes.byref(h), ctypes.byref(f), table_begin, tc,
                                             keys.data_ptr(), sigs.data_ptr() if with_values else None))
        return (keys, sigs) if with_values else keys

    def _outputs(self, cap):
        dev = torch.device("cuda", self.device)
        return (torch.empty(cap, dtype=torch.int32, device=dev), torch.empty(cap, dtype=torch.int32, device=dev),
                torch.empty(cap, dtype=torch.uint8, device=dev))

    def _refetch(self, rc, total, capacity):
        """After E_CAPACITY with automatic capacity: fetch the kept result."""
        oi, oj, ov = self._outputs(max(total, 1))
        if rc == E_CAPACITY and capacity is None:
            rc = library().fast_lsh_copy_result(self._ctx, oi.data_ptr(), oj.data_ptr(), ov.data_ptr(), total)
        return rc, (oi, oj, ov)

    def search(self, rows, dim, t, r, scheme, a, b, min_lag, min_votes, occ_num=0, occ_den=0,
               want_distinct=False, capacity: int | None = None, graph=False):
        """Sorted (i, j, votes) CUDA tensors (int32, int32, uint8) and Stats."""
        h, keep = _hash_struct(dim, t, r, scheme, a, b)
        f, keep2 = _fps_struct(rows)
        flt = Filter(min_lag, min_votes, occ_num, occ_den)
        flags = (WANT_DISTINCT if want_distinct else 0) | (USE_GRAPH if graph else 0)
        cap = max(1, f.n // 4) if capacity is None else capacity
        oi, oj, ov = self._outputs(cap)
        st = _Stats()
        rc = library().fast_lsh_search_ex(self._ctx, ctypes.byref(h), ctypes.byref(f), ctypes.byref(flt), flags,
                                          oi.data_ptr(), oj.data_ptr(), ov.data_ptr(), cap, ctypes.byref(st))
        if rc == E_CAPACITY and capacity is None:
            rc, (oi, oj, ov) = self._refetch(rc, st.n_out, capacity)
        _check(rc)
        m = st.n_out
        stats = Stats(*[int(getattr(st, k)) for k, _ in _Stats._fields_])
        return oi[:m], oj[:m], ov[:m], stats

    def search_bounded(self, rows, dim, t, r, scheme, a, b, min_lag, min_votes, occ_num=0, occ_den=0,
                       group_tables=10, want_distinct=False, capacity: int | None = None):
        """The search with tables taken group_tables at a time (same output)."""
        h, keep = _hash_struct(dim, t, r, scheme, a, b)
        f, keep2 = _fps_struct(rows)
        flt = Filter(min_lag, min_votes, occ_num, occ_den)
        flags = WANT_DISTINCT if want_distinct else 0
        cap = max(1, f.n // 4) if capacity is None else capacity
        oi, oj, ov = self._outputs(cap)
        st = _Stats()
        rc = library().fast_lsh_search_bounded(self._ctx, ctypes.byref(h), ctypes.byref(f), ctypes.byref(flt),
                                               flags, group_tables, oi.data_ptr(), oj.data_ptr(), ov.data_ptr(),
                                               cap, ctypes.byref(st))
        if rc == E_CAPACITY and capacity is None:
            rc, (oi, oj, ov) = self._refetch(rc, st.n_out, capacity)
        _check(rc)
        m = st.n_out
        stats = Stats(*[int(getattr(st, k)) for k, _ in _Stats._fields_])
        return oi[:m], oj[:m], ov[:m], stats

    def search_batched(self, stations, dim, t, r, scheme, a, b, min_lag, min_votes, occ_num=0, occ_den=0,
                       want_distinct=False, capacity: int | None = None, graph=False):
        """One search over several stations.  Returns (i, j, votes, offsets,
        [Stats per station]): station s owns entries offsets[s]:offsets[s+1]
        of the CUDA tensors, with station-local ids."""
        S = len(stations)
        h, keep = _hash_struct(dim, t, r, scheme, a, b)
        fl = [_fps_struct(x) for x in stations]
        fa = (Fps * max(S, 1))(*[x[0] for x in fl])
        flt = Filter(min_lag, min_votes, occ_num, occ_den)
        flags = (WANT_DISTINCT if want_distinct else 0) | (USE_GRAPH if graph else 0)
        total = sum(x[0].n for x in fl)
        cap = max(1, total // 4) if capacity is None else capacity
        oi, oj, ov = self._outputs(cap)
        offs = (_u64 * (S + 1))()
        sts = (_Stats * max(S, 1))()
        rc = library().fast_lsh_search_batched(self._ctx, ctypes.byref(h), S, fa, ctypes.byref(flt), flags,
                                               oi.data_ptr(), oj.data_ptr(), ov.data_ptr(), cap, offs, sts)
        if rc == E_CAPACITY and capacity is None:
            rc, (oi, oj, ov) = self._refetch(rc, int(offs[S]), capacity)
        _check(rc)
        m = int(offs[S])
        stats = [Stats(*[int(getattr(sts[k], f)) for f, _ in _Stats._fields_]) for k in range(S)]
        return oi[:m], oj[:m], ov[:m], np.array(list(offs), dtype=np.int64), stats


# ---------------------------------------------------------------------------
# Serving form
# ---------------------------------------------------------------------------
class ServerConfig(ctypes.Structure):
    _fields_ = [("max_batch", _u32), ("max_chunk", _u32), ("delta_rows", _u64), ("slack_rows", _u64),
                ("hbm_budget", _u64)]


class _ServerState(ctypes.Structure):
    _fields_ = [("stations", _u32), ("waiting", _u32), ("resident_bytes", _u64), ("workspace_bytes", _u64),
                ("batches", _u64), ("chunks", _u64), ("largest_batch", _u64)]


def _server_lib():
    lib = library()
    if not getattr(lib, "_server_ready", False):
        lib.fast_lsh_server_create.argtypes = [_i32, ctypes.POINTER(Hash), ctypes.POINTER(Filter),
                                               ctypes.POINTER(ServerConfig), ctypes.POINTER(_vp)]
        lib.fast_lsh_server_destroy.argtypes = [_vp]
        lib.fast_lsh_server_add_station.argtypes = [_vp, ctypes.POINTER(Fps), ctypes.POINTER(_u32)]
        lib.fast_lsh_server_submit.argtypes = [_vp, _u32, ctypes.POINTER(Fps), _u64, ctypes.POINTER(_u64)]
        lib.fast_lsh_server_poll.argtypes = [_vp, _u64, _i32, ctypes.POINTER(_Stats), ctypes.POINTER(_u64)]
        lib.fast_lsh_server_take.argtypes = [_vp, _u64, _vp, _vp, _vp, _u64]
        lib.fast_lsh_server_now_ns.argtypes = [_vp]
        lib.fast_lsh_server_now_ns.restype = _u64
        lib.fast_lsh_server_info.argtypes = [_vp, ctypes.POINTER(_ServerState)]
        lib.fast_lsh_plan_batch.argtypes = [_vp, _u32, _u32, _vp, ctypes.POINTER(_u32)]
        lib._server_ready = True
    return lib


def plan_batch(stations, max_batch: int):
    """Indices of the waiting chunks (stations[k] = station of the k-th,
    oldest first) that the next batch takes (host-side rule)."""
    st = np.ascontiguousarray(stations, dtype=np.uint32)
    picked = np.empty(max(len(st), 1), dtype=np.uint32)
    n = _u32()
    _check(_server_lib().fast_lsh_plan_batch(st.ctypes.data, len(st), max_batch, picked.ctypes.data,
                                             ctypes.byref(n)))
    return picked[: n.value].tolist()


class Server:
    """Stations with resident tables, searched chunk by chunk (continuous
    batching on a worker thread of the library)."""

    def __init__(self, dim, t, r, scheme, a, b, min_lag, min_votes, device=0, max_batch=8, max_chunk=3600,
                 delta_rows=262144, slack_rows=2_000_000, hbm_budget=0):
        lib = _server_lib()
        h, self._keep = _hash_struct(dim, t, r, scheme, a, b)
        cfg = ServerConfig(max_batch, max_chunk, delta_rows, slack_rows, hbm_budget)
        flt = Filter(min_lag, min_votes, 0, 0)
        sv = _vp()
        _check(lib.fast_lsh_server_create(device, ctypes.byref(h), ctypes.byref(flt), ctypes.byref(cfg),
                                          ctypes.byref(sv)))
        self._sv = sv
        self._rows = {}  # ticket -> device rows kept alive until the chunk is done

    def close(self):
        if getattr(self, "_sv", None):
            _server_lib().fast_lsh_server_destroy(self._sv)
            self._sv = None
            self._rows.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def add_station(self, rows) -> int:
        f, keep = _fps_struct(rows)
        st = _u32()
        _check(_server_lib().fast_lsh_server_add_station(self._sv, ctypes.byref(f), ctypes.byref(st)))
        return int(st.value)

    def now_ns(self) -> int:
        return int(_server_lib().fast_lsh_server_now_ns(self._sv))

    def submit(self, station: int, rows, arrival_ns: int | None = None) -> int:
        f, keep = _fps_struct(rows)
        tk = _u64()
        arr = self.now_ns() if arrival_ns is None else arrival_ns
        _check(_server_lib().fast_lsh_server_submit(self._sv, station, ctypes.byref(f), arr, ctypes.byref(tk)))
        self._rows[int(tk.value)] = keep
        return int(tk.value)

    def poll(self, ticket: int, wait: bool = False):
        """None while the chunk waits or runs; else (Stats, done_ns)."""
        st = _Stats()
        done = _u64()
        rc = _server_lib().fast_lsh_server_poll(self._sv, ticket, 1 if wait else 0, ctypes.byref(st),
                                                ctypes.byref(done))
        if rc == E_BUSY:
            return None
        if rc != OK:
            self._rows.pop(ticket, None)
        _check(rc)
        return Stats(*[int(getattr(st, k)) for k, _ in _Stats._fields_]), int(done.value)

    def take(self, ticket: int):
        """(i, j, votes) numpy arrays of a done chunk; releases the ticket."""
        st, _ = self.poll(ticket, wait=True)
        m = st.n_out
        oi = np.empty(max(m, 1), np.uint32)
        oj = np.empty(max(m, 1), np.uint32)
        ov = np.empty(max(m, 1), np.uint8)
        _check(_server_lib().fast_lsh_server_take(self._sv, ticket, oi.ctypes.data, oj.ctypes.data, ov.ctypes.data,
                                                  m))
        self._rows.pop(ticket, None)
        return oi[:m], oj[:m], ov[:m]

    def info(self) -> dict:
        s = _ServerState()
        _check(_server_lib().fast_lsh_server_info(self._sv, ctypes.byref(s)))
        return {k: int(getattr(s, k)) for k, _ in _ServerState._fields_}
