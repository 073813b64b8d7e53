"""Pins of the oracle's fingerprint extraction (section 5): the Haar
transform against hand-worked values and an independently built Haar matrix;
the spectrogram against closed forms for pure tones and a direct DFT sum;
spectral-image averaging, median / MAD and the top-K sign code on hand-built
cases; fingerprints of repeated events."""
import numpy as np
import pytest

import synth
from oracle import fingerprint as fp

P = fp.FpParams()


def haar_matrix(n):
    """Orthonormal Haar matrix from its recursion: the first half applies
    H_{n/2} to pairwise sums, the second half gives the finest differences."""
    if n == 1:
        return np.ones((1, 1))
    h = haar_matrix(n // 2)
    s = np.sqrt(0.5)
    top = np.kron(h, np.array([[1.0, 1.0]])) * s
    bot = np.kron(np.eye(n // 2), np.array([[1.0, -1.0]])) * s
    return np.vstack([top, bot])


def test_haar_hand_worked():
    # [4, 2, 5, 5]: sums (6, 10)/sqrt2, details (2, 0)/sqrt2; then 16/2 = 8, (6 - 10)/2 = -2
    got = fp.haar1d(np.array([4.0, 2.0, 5.0, 5.0]))
    assert np.allclose(got, [8.0, -2.0, np.sqrt(2.0), 0.0], atol=1e-12)
    assert np.allclose(fp.haar1d(np.ones(8)), [np.sqrt(8.0)] + [0.0] * 7, atol=1e-12)


@pytest.mark.parametrize("n", [2, 8, 64])
def test_haar_matches_matrix(n):
    rng = np.random.default_rng(n)
    v = rng.normal(size=(5, n))
    h = haar_matrix(n)
    assert np.allclose(fp.haar1d(v), v @ h.T, atol=1e-12)
    assert np.allclose(h @ h.T, np.eye(n), atol=1e-12)  # orthonormal: energy preserved


def test_haar2d_matches_kronecker():
    rng = np.random.default_rng(3)
    img = rng.normal(size=(P.rows, P.cols))
    want = haar_matrix(P.rows) @ img @ haar_matrix(P.cols).T
    assert np.allclose(fp.haar2d(img), want, atol=1e-10)
    assert np.isclose((fp.haar2d(img) ** 2).sum(), (img ** 2).sum())


def test_spectrogram_pure_tone_closed_form():
    # cos(2 pi k0 n / L) under the periodic Hann window: bin k0 holds L/4,
    # bins k0 +- 1 hold L/8, every other bin 0
    k0 = 10
    n = np.arange(5000)
    x = np.cos(2.0 * np.pi * k0 * n / P.window)
    s = fp.spectrogram(x, P)
    b = k0 - P.band_lo
    assert np.allclose(s[:, b], (P.window / 4) ** 2) and np.allclose(s[:, b - 1], (P.window / 8) ** 2)
    assert np.allclose(s[:, b + 1], (P.window / 8) ** 2)
    others = np.delete(s, [b - 1, b, b + 1], axis=1)
    assert np.abs(others).max() < 1e-9


def test_spectrogram_direct_dft():
    rng = np.random.default_rng(4)
    x = rng.normal(size=1000)
    s = fp.spectrogram(x, P)
    w = fp.hann(P)
    for f in (0, 37, fp.n_frames(len(x), P) - 1):
        seg = x[f * P.hop:f * P.hop + P.window] * w
        for k in (P.band_lo, 20, P.band_hi - 1):
            re = sum(seg[m] * np.cos(2 * np.pi * k * m / P.window) for m in range(P.window))
            im = sum(seg[m] * np.sin(2 * np.pi * k * m / P.window) for m in range(P.window))
            assert np.isclose(s[f, k - P.band_lo], re * re + im * im, rtol=1e-10)


def test_image_averages_frame_pairs():
    spec = np.arange(300 * P.rows, dtype=np.float64).reshape(300, P.rows)
    img = fp.image(spec, 3, P)
    f0 = 3 * P.fp_lag
    assert img.shape == (P.rows, P.cols)
    assert np.allclose(img[:, 5], (spec[f0 + 10] + spec[f0 + 11]) / 2)
    assert fp.n_frames(1000, P) == 81 and fp.n_fingerprints(1000, P) == 0
    assert fp.n_fingerprints(P.window + (P.fp_frames - 1) * P.hop, P) == 1
    assert fp.n_fingerprints(100 * 3600, P) == 3586  # one hour at 100 Hz: 35,981 frames


def test_median_mad_and_sign_code():
    v = np.array([[1.0], [5.0], [3.0], [2.0], [4.0], [9.0]])
    med, mad = fp.median_mad(v)  # sorted 1 2 3 4 5 9: lower median 3; |dev| 0 1 1 2 2 6: lower median 1
    assert med[0] == 3.0 and mad[0] == 1.0
    z = np.array([[0.5, -3.0, 0.0, 3.0, -0.1, 2.0]])
    # top 3 by |z|: c=1 (-3), c=3 (3) tie broken by index, then c=5 (2)
    assert fp.top_binarize(z, 3)[0].tolist() == [3, 6, 10]
    # zeros are never chosen: K = 6 gives the five non-zero coefficients
    assert fp.top_binarize(z, 6)[0].tolist() == [0, 3, 6, 9, 10]
    coef = np.array([[1.0, 7.0], [3.0, 7.0], [5.0, 7.0]])
    m, d = fp.median_mad(coef)
    assert np.array_equal(fp.normalize(coef, m, d), [[-1.0, 0.0], [0.0, 0.0], [1.0, 0.0]])  # MAD 0: z = 0


def test_fingerprints_of_identical_windows():
    # a noise record repeating every 1500 samples: fingerprints 15 apart
    # (1500 samples at a 100-sample lag) see identical samples
    rng = np.random.default_rng(5)
    x = np.tile(rng.normal(size=1500), 40)
    nf = fp.n_fingerprints(len(x), P)
    fps, z, med, mad = fp.fingerprints(x, P, np.arange(0, nf, 3), np.arange(nf))
    assert all(len(f) == P.top_k for f in fps)
    assert all(np.array_equal(fps[i], fps[i + 15]) for i in range(nf - 15))
    assert not np.array_equal(fps[0], fps[1])
    assert all((f < P.dim).all() and (np.diff(f.astype(np.int64)) > 0).all() for f in fps)


def test_fingerprints_noisy_copies_are_similar():
    spec = synth.WaveSpec(n=100 * 3600, seed=6, n_sources=6, rep_min=4, rep_max=4, noise_std=1.0, amp_lo=6.0,
                          amp_hi=10.0)
    x, starts, src = synth.waveform(spec, events=True)
    nf = fp.n_fingerprints(len(x), P)
    fps, _, _, _ = fp.fingerprints(x, P, np.arange(0, nf, 5), np.arange(nf))
    jac = lambda a, b: len(np.intersect1d(a, b)) / len(np.union1d(a, b))
    ev = {}
    for s0, s in zip(starts.tolist(), src.tolist()):
        ev.setdefault(s, []).append(s0 // 100 + 4)
    copies = [jac(fps[a], fps[b]) for ids in ev.values() for a in ids for b in ids if a < b]
    rng = np.random.default_rng(0)
    rand = [jac(fps[a], fps[b]) for a, b in rng.integers(0, nf, (200, 2)) if abs(a - b) > 20]
    assert np.mean(copies) > 0.3 and np.mean(rand) < 0.1
