"""Seeded inputs for the spatiotemporal-alignment tests: channel search
outputs and (dt, idx1)-ordered entries.  Input generation only (no merge,
no clustering arithmetic)."""
from __future__ import annotations

import numpy as np


def channels(seed, n_ch=3, n=400, pairs=300, shared=0.4, vmax=12):
    """n_ch channels' search outputs over n fingerprints ((i, j, votes),
    i < j, sorted by (i, j), no repeats): a share of the pairs appears in
    every channel, each channel with its own votes."""
    rng = np.random.default_rng(seed)

    def draw(k):
        i = rng.integers(0, n - 1, k)
        j = i + 1 + (rng.random(k) * (n - 1 - i)).astype(np.int64)
        return np.unique((i.astype(np.uint64) << np.uint64(32)) | j.astype(np.uint64))

    common = draw(int(pairs * shared))
    out = []
    for _ in range(n_ch):
        key = np.union1d(common, draw(pairs - len(common)))
        i = (key >> np.uint64(32)).astype(np.uint32)
        j = (key & np.uint64(0xFFFFFFFF)).astype(np.uint32)
        v = rng.integers(1, vmax + 1, len(key)).astype(np.uint8)
        out.append((i, j, v))
    return out


def entries(seed, n_diag=12, streaks=6, noise=120, span=400, dt0=5, streak_len=(3, 25), step=(1, 4)):
    """(dt, idx1, sim) strictly ordered by (dt, idx1): thin diagonal streaks
    (runs with small gaps, some entries spilling onto a neighbouring
    diagonal) among isolated points."""
    rng = np.random.default_rng(seed)
    d_all, x_all = [], []
    for _ in range(streaks):
        d0, x0 = int(rng.integers(dt0, dt0 + n_diag)), int(rng.integers(0, span))
        k = int(rng.integers(streak_len[0], streak_len[1]))
        x = x0 + np.cumsum(rng.integers(step[0], step[1], k))
        d = d0 + np.where(rng.random(k) < 0.3, rng.integers(-1, 2, k), 0)
        d_all.append(np.maximum(d, 1))
        x_all.append(x)
    d_all.append(rng.integers(dt0, dt0 + n_diag, noise))
    x_all.append(rng.integers(0, span, noise))
    d = np.concatenate(d_all).astype(np.uint64)
    x = np.concatenate(x_all).astype(np.uint64)
    key = np.unique((d << np.uint64(32)) | x)
    sim = rng.integers(1, 20, len(key)).astype(np.uint32)
    return (key >> np.uint64(32)).astype(np.uint32), (key & np.uint64(0xFFFFFFFF)).astype(np.uint32), sim
