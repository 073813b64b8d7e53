"""Seeded synthetic fingerprint workloads shared by the oracle and the GPU path.

The arithmetic lives in ``synth.c`` (compiled to ``libsynth.so``); this module
only marshals arguments.  Nothing here computes signatures, buckets or votes.

Workload recipes (sizes, seeds and structure of each configuration) are named
after what they model:

* ``tiny_uniform``   20,000 independent uniform 200-of-4096 fingerprints with
                     50 events copied into 5 slots each, every copy keeping
                     160 of the template's 200 bits.
* ``station``        one station at a 1 s lag: a Markov background in which
                     each fingerprint keeps 140 of the previous one's 200
                     bits, plus repeating sources with 3-40 copies whose
                     Jaccard similarity to the template is drawn from
                     U[0.4, 0.9] per copy.  90 days = 7,776,000 rows.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading
from dataclasses import dataclass, replace

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "libsynth.so")
_SRC = os.path.join(_HERE, "synth.c")


def build() -> str:
    """Compile ``libsynth.so`` in place (always recompiles)."""
    tmp = _SO + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-std=c11", _SRC, "-o", tmp, "-lm"])
    os.replace(tmp, _SO)
    return _SO


class _Spec(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_uint64),
        ("dim", ctypes.c_uint32),
        ("nnz", ctypes.c_uint32),
        ("seed", ctypes.c_uint64),
        ("markov_keep", ctypes.c_uint32),
        ("n_sources", ctypes.c_uint32),
        ("rep_min", ctypes.c_uint32),
        ("rep_max", ctypes.c_uint32),
        ("plant_keep", ctypes.c_uint32),
        ("jac_lo_milli", ctypes.c_uint32),
        ("jac_hi_milli", ctypes.c_uint32),
        ("noise_permille", ctypes.c_uint32),
        ("noise_keep", ctypes.c_uint32),
        ("chain_len", ctypes.c_uint64),
        ("channel", ctypes.c_uint32),
    ]


class _WaveSpec(ctypes.Structure):
    _fields_ = [("n", ctypes.c_uint64), ("seed", ctypes.c_uint64), ("n_sources", ctypes.c_uint32),
                ("rep_min", ctypes.c_uint32), ("rep_max", ctypes.c_uint32), ("event_len", ctypes.c_uint32),
                ("noise_std", ctypes.c_float), ("amp_lo", ctypes.c_float), ("amp_hi", ctypes.c_float),
                ("reserved", ctypes.c_uint32)]


_LIB = None
_LOCK = threading.Lock()


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
        lib.synth_generate_range.argtypes = [ctypes.POINTER(_Spec), ctypes.c_uint64, ctypes.c_uint64,
                                             ctypes.c_void_p, ctypes.c_void_p]
        lib.synth_generate_range.restype = ctypes.c_int
        lib.synth_planted_count.argtypes = [ctypes.POINTER(_Spec)]
        lib.synth_waveform_range.argtypes = [ctypes.POINTER(_WaveSpec), ctypes.c_uint64, ctypes.c_uint64,
                                             ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
        lib.synth_waveform_range.restype = ctypes.c_int
        lib.synth_wave_events.argtypes = [ctypes.POINTER(_WaveSpec)]
        lib.synth_wave_events.restype = ctypes.c_uint64
        lib.synth_planted_count.restype = ctypes.c_uint64
        _LIB = lib
    return _LIB


@dataclass(frozen=True)
class Spec:
    n: int
    dim: int = 4096
    nnz: int = 200
    seed: int = 0
    markov_keep: int = 0
    n_sources: int = 0
    rep_min: int = 1
    rep_max: int = 1
    plant_keep: int = 0
    jac_lo_milli: int = 0
    jac_hi_milli: int = 0
    noise_permille: int = 0
    noise_keep: int = 0
    chain_len: int = 0
    channel: int = 0

    def _c(self) -> _Spec:
        return _Spec(*[getattr(self, f) for f, _ in _Spec._fields_])


def generate(spec: Spec, lo: int = 0, hi: int | None = None, labels: bool = False, out: np.ndarray | None = None):
    """Rows [lo, hi) of ``spec`` as a C-ordered ``uint16[hi-lo, nnz]`` array
    (sorted indices per row); with ``labels`` also ``int32[hi-lo]`` holding -1
    (background), the planted source id, or -2 (noise copy).  ``out``: an
    existing C-ordered 2-byte array of that shape to fill instead."""
    hi = spec.n if hi is None else hi
    if out is not None:
        assert out.flags.c_contiguous and out.itemsize == 2 and out.shape == (hi - lo, spec.nnz)
        rows = out
    else:
        rows = np.empty((hi - lo, spec.nnz), dtype=np.uint16)
    lab = np.empty(hi - lo, dtype=np.int32) if labels else None
    c = spec._c()
    rc = _lib().synth_generate_range(ctypes.byref(c), lo, hi, rows.ctypes.data,
                                     lab.ctypes.data if labels else None)
    if rc == 3:
        raise MemoryError(f"synth: a host allocation failed while generating rows [{lo}, {hi}) of {spec}")
    if rc != 0:
        raise ValueError(f"synth: invalid spec {spec} (code {rc})")
    return (rows, lab) if labels else rows


def planted_count(spec: Spec) -> int:
    c = spec._c()
    return int(_lib().synth_planted_count(ctypes.byref(c)))


# --------------------------------------------------------------------------
# Workload recipes
# --------------------------------------------------------------------------
DAY = 86_400
STATION_90D = 90 * DAY          # 7,776,000 fingerprints at a 1 s lag
STATION_180D = 180 * DAY        # 15,552,000
STATION_5Y = 157_788_000        # 5 x 365.25 days
CHUNK = 3_600                   # one hour of fingerprints at a 1 s lag
BATCH_LENGTHS_M = (1, 2, 3, 4, 5, 6, 7, 8, 10, 12, 14, 16)


def tiny_uniform(n: int = 20_000, seed: int = 101) -> Spec:
    """Independent uniform background with 50 events x 5 copies keeping 80 %."""
    return Spec(n=n, seed=seed, n_sources=50, rep_min=5, rep_max=5, plant_keep=160)


def station(n: int = STATION_90D, seed: int = 102, sources_per_90d: int = 2000) -> Spec:
    """Markov background (70 % kept) with repeating sources, J ~ U[0.4, 0.9].
    The source count scales with length (2,000 per 90 days by default)."""
    ns = max(1, round(sources_per_90d * n / STATION_90D))
    return Spec(n=n, seed=seed, markov_keep=140, n_sources=ns, rep_min=3, rep_max=40,
                jac_lo_milli=400, jac_hi_milli=900)


def long_station(n: int = STATION_5Y, seed: int = 105, n_sources: int = 20_000,
                 chain_len: int = 1_000_000) -> Spec:
    """Five years at a 1 s lag: Markov background (70 % kept) in independent
    chains of ``chain_len`` rows (so that generation runs in parallel), with
    ``n_sources`` repeating sources, J ~ U[0.4, 0.9]."""
    return Spec(n=n, seed=seed, markov_keep=140, n_sources=n_sources, rep_min=3, rep_max=40,
                jac_lo_milli=400, jac_hi_milli=900, chain_len=chain_len)


def with_noise(spec: Spec, permille: int = 50, keep: int = 190) -> Spec:
    """Test-only variant: a repeating-noise source fills `permille` of all
    slots with copies keeping `keep` of its bits (drives the occurrence filter)."""
    return replace(spec, noise_permille=permille, noise_keep=keep)


# --------------------------------------------------------------------------
# Continuous waveforms (input of the fingerprint extraction)
# --------------------------------------------------------------------------
@dataclass(frozen=True)
class WaveSpec:
    """One channel sampled at 100 Hz: Gaussian noise of noise_std plus
    n_sources repeating sources (rep_min..rep_max events each, event_len
    samples, a P and an S wave packet, amplitude ~ U[amp_lo, amp_hi])."""
    n: int
    seed: int = 0
    n_sources: int = 0
    rep_min: int = 1
    rep_max: int = 1
    event_len: int = 1500
    noise_std: float = 1.0
    amp_lo: float = 2.0
    amp_hi: float = 8.0

    def _c(self) -> _WaveSpec:
        return _WaveSpec(self.n, self.seed, self.n_sources, self.rep_min, self.rep_max, self.event_len,
                         self.noise_std, self.amp_lo, self.amp_hi, 0)


def waveform(spec: WaveSpec, lo: int = 0, hi: int | None = None, events: bool = False, out: np.ndarray | None = None):
    """Samples [lo, hi) as float32 (and, with ``events``, every event's
    (start sample, source) arrays)."""
    hi = spec.n if hi is None else hi
    x = out if out is not None else np.empty(hi - lo, dtype=np.float32)
    assert x.dtype == np.float32 and x.flags.c_contiguous and len(x) == hi - lo
    c = spec._c()
    ne = int(_lib().synth_wave_events(ctypes.byref(c)))
    st = np.empty(max(ne, 1), dtype=np.uint64) if events else None
    so = np.empty(max(ne, 1), dtype=np.uint32) if events else None
    rc = _lib().synth_waveform_range(ctypes.byref(c), lo, hi, x.ctypes.data, st.ctypes.data if events else None,
                                     so.ctypes.data if events else None)
    if rc == 3:
        raise MemoryError("synth: a host allocation failed")
    if rc != 0:
        raise ValueError(f"synth: invalid waveform spec {spec} (code {rc})")
    return (x, st[:ne], so[:ne]) if events else x


def station_waveform(days: float = 90, seed: int = 402, sources_per_90d: int = 2000) -> WaveSpec:
    """A station's continuous record at 100 Hz with repeating sources (3-40
    events each), the waveform counterpart of ``station``."""
    n = int(round(days * DAY * 100))
    ns = max(1, round(sources_per_90d * days / 90))
    return WaveSpec(n=n, seed=seed, n_sources=ns, rep_min=3, rep_max=40)
