"""CPU ORACLE — TEST INFRASTRUCTURE ONLY: fingerprint extraction (section 5).

A plain float64 numpy implementation of the steps section 5.1 lists, in its
order, for one channel of continuous data:

1. Spectrogram: power of the short-time Fourier transform (periodic Hann
   window of ``window`` samples, frames every ``hop`` samples), the
   frequency bins [band_lo, band_hi) kept (the spectrogram cut at the
   corners of the bandpass filter, section 6.5); each fingerprint takes
   ``fp_frames`` consecutive frames, every ``fp_lag`` frames, and smooths
   them into a spectral image of fixed size by averaging ``time_ds``
   consecutive frames (rows: frequency bins, columns: time).
2. Wavelet transform: the two-dimensional orthonormal Haar transform of the
   image (the standard decomposition: the full one-dimensional transform of
   every row, then of every column; coefficient order per axis: the final
   average, then the details from the coarsest level to the finest).
3. Normalization: each coefficient c is replaced by (w_c - median_c) / MAD_c,
   with the median and the median absolute deviation of coefficient c over
   a sample of the fingerprints (section 5.2: statistics from a random
   sample; the sample's indices are an input).  Median of m values: the
   lower middle one, sorted[(m - 1) // 2].  MAD_c = 0: the coefficient's z
   is 0.
4. Top coefficients: the K coefficients of largest |z| (ties: the smaller
   coefficient index first); only z != 0 can be chosen.
5. Binarize: coefficient c with z > 0 sets bit 2c, z < 0 sets bit 2c + 1
   (the paper's 2-bit sign code: 1 -> 10, -1 -> 01, 0 -> 00); a fingerprint
   is the sorted list of its set bits, of dimension 2 * (image size).

Readings where the paper is silent (window, hop, band, image size, K, Hann
form, median of an even count, MAD = 0) are the parameters above, chosen so
that the default yields 4096-dimensional fingerprints with K = 200 set bits
at a 1 s lag of 100 Hz data, the fingerprints the search is run on.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass(frozen=True)
class FpParams:
    window: int = 200      # samples per STFT frame (2 s at 100 Hz)
    hop: int = 10          # samples between frames (0.1 s)
    band_lo: int = 4       # first frequency bin kept (2 Hz)
    band_hi: int = 36      # one past the last bin kept (18 Hz): 32 rows
    fp_frames: int = 128   # frames per fingerprint (12.8 s)
    time_ds: int = 2       # frames averaged per image column: 64 columns
    fp_lag: int = 10       # frames between fingerprints (1 s)
    top_k: int = 200

    @property
    def rows(self) -> int:
        return self.band_hi - self.band_lo

    @property
    def cols(self) -> int:
        return self.fp_frames // self.time_ds

    @property
    def dim(self) -> int:
        return 2 * self.rows * self.cols


def n_frames(n_samples: int, p: FpParams) -> int:
    return 0 if n_samples < p.window else (n_samples - p.window) // p.hop + 1


def n_fingerprints(n_samples: int, p: FpParams) -> int:
    f = n_frames(n_samples, p)
    return 0 if f < p.fp_frames else (f - p.fp_frames) // p.fp_lag + 1


def hann(p: FpParams) -> np.ndarray:
    n = np.arange(p.window)
    return 0.5 * (1.0 - np.cos(2.0 * np.pi * n / p.window))


def spectrogram(x: np.ndarray, p: FpParams, f0: int = 0, f1: int | None = None) -> np.ndarray:
    """Power of frames [f0, f1) in the kept band: float64 [frames, rows]."""
    f1 = n_frames(len(x), p) if f1 is None else f1
    if f1 <= f0:
        return np.zeros((0, p.rows))
    idx = (np.arange(f0, f1) * p.hop)[:, None] + np.arange(p.window)[None, :]
    frames = np.asarray(x, dtype=np.float64)[idx] * hann(p)[None, :]
    spec = np.fft.rfft(frames, axis=1)[:, p.band_lo:p.band_hi]
    return spec.real ** 2 + spec.imag ** 2


def image(spec: np.ndarray, i: int, p: FpParams, frame0: int = 0) -> np.ndarray:
    """Spectral image of fingerprint i (float64 [rows, cols]) from the
    spectrogram whose first row is frame `frame0`."""
    a = i * p.fp_lag - frame0
    block = spec[a:a + p.fp_frames]  # [fp_frames, rows]
    return block.reshape(p.cols, p.time_ds, p.rows).mean(axis=1).T


def haar1d(v: np.ndarray) -> np.ndarray:
    """Full orthonormal Haar transform along the last axis (length 2^m):
    [final average, details coarsest .. finest]."""
    out = np.array(v, dtype=np.float64)
    n = out.shape[-1]
    s = np.sqrt(0.5)
    while n > 1:
        a = (out[..., 0:n:2] + out[..., 1:n:2]) * s
        d = (out[..., 0:n:2] - out[..., 1:n:2]) * s
        out[..., : n // 2] = a
        out[..., n // 2:n] = d
        n //= 2
    return out


def haar2d(img: np.ndarray) -> np.ndarray:
    """Standard 2-D decomposition: every row, then every column."""
    return haar1d(haar1d(img).swapaxes(-1, -2)).swapaxes(-1, -2)


def coefficients(x: np.ndarray, p: FpParams, ids=None, frame0: int = 0) -> np.ndarray:
    """Haar coefficients (float64 [len(ids), rows * cols]) of fingerprints ids
    (default: all) of the samples x, whose first sample is frame frame0's."""
    nf = n_fingerprints(len(x) + frame0 * p.hop, p)
    ids = np.arange(nf) if ids is None else np.asarray(ids)
    out = np.empty((len(ids), p.rows * p.cols))
    for k, i in enumerate(ids):
        f0 = int(i) * p.fp_lag - frame0
        spec = spectrogram(x, p, f0, f0 + p.fp_frames)
        out[k] = haar2d(image(spec, int(i), p, frame0=f0 + frame0)).reshape(-1)
    return out


def lower_median(v: np.ndarray, axis: int = 0) -> np.ndarray:
    s = np.sort(v, axis=axis)
    m = s.shape[axis]
    return np.take(s, (m - 1) // 2, axis=axis)


def median_mad(coef_sample: np.ndarray):
    """Per coefficient: the lower median and the MAD over the sample rows."""
    med = lower_median(coef_sample, axis=0)
    mad = lower_median(np.abs(coef_sample - med[None, :]), axis=0)
    return med, mad


def normalize(coef: np.ndarray, med: np.ndarray, mad: np.ndarray) -> np.ndarray:
    z = np.zeros_like(coef)
    ok = mad > 0
    z[:, ok] = (coef[:, ok] - med[None, ok]) / mad[None, ok]
    return z


def top_binarize(z: np.ndarray, k: int):
    """Per row: the sorted set bits (list of uint16 arrays) of the K
    coefficients of largest |z| (ties: smaller index), z != 0 only."""
    out = []
    for row in z:
        order = np.lexsort((np.arange(len(row)), -np.abs(row)))  # |z| descending, index ascending
        pick = [c for c in order[:k] if row[c] != 0]
        bits = sorted(2 * c + (1 if row[c] < 0 else 0) for c in pick)
        out.append(np.array(bits, dtype=np.uint16))
    return out


def fingerprints(x: np.ndarray, p: FpParams, sample_ids, ids=None):
    """Fingerprints (list of sorted uint16 arrays) of fingerprints ids (default
    all) of x, normalized with the statistics of fingerprints sample_ids.
    Also returns (z, med, mad) for the checks."""
    med, mad = median_mad(coefficients(x, p, sample_ids))
    z = normalize(coefficients(x, p, ids), med, mad)
    return top_binarize(z, p.top_k), z, med, mad
