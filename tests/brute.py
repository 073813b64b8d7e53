"""Brute-force references for tiny inputs (pure Python / numpy).

These take a different route from the oracle so that they can pin it:
signatures are found by evaluating every hash on every set element with
Python integers, and the search compares every pair of fingerprints in every
table (O(N^2 t)) instead of grouping by bucket.
"""
from __future__ import annotations

from collections import Counter

import numpy as np

P = 2**31 - 1


def keys_brute(rows, dim, t, r, scheme, a, b):
    """Band keys uint64[t, n] by direct evaluation (scheme 0 MinHash, 1 Min-Max)."""
    bits = max(0, (dim - 1).bit_length())
    n = len(rows)
    keys = np.zeros((t, n), dtype=np.uint64)
    for i, row in enumerate(rows):
        xs = [int(x) for x in row]
        for u in range(t):
            arg = []
            for s in range(r):
                if scheme == 0:
                    f, want_max = u * r + s, False
                else:
                    f, want_max = u * (r // 2) + s // 2, bool(s & 1)
                vals = [((int(a[f]) * x + int(b[f])) % P, x) for x in xs]
                best = max(vals) if want_max else min(vals)
                arg.append(best[1])
            assert bits * r <= 64
            k = 0
            for s, x in enumerate(arg):
                k |= x << (bits * s)
            keys[u, i] = k
    return keys


def search_brute(keys, min_lag, min_votes, occ_num=0, occ_den=0):
    """All-pairs reference: returns (list of (i, j, votes), stats dict, flags)."""
    keys = np.asarray(keys)
    t, n = keys.shape
    flags = np.zeros(n, dtype=bool)
    max_bucket = 0
    for u in range(t):
        cnt = Counter(keys[u].tolist())
        if cnt:
            max_bucket = max(max_bucket, max(cnt.values()))
        if occ_den:
            for i in range(n):
                if cnt[keys[u, i]] * occ_den > n * occ_num:
                    flags[i] = True
    out = []
    e_raw = e_voted = n_distinct = 0
    for i in range(n):
        eq = (keys[:, i + 1:] == keys[:, i:i + 1]).sum(axis=0)
        e_raw += int(eq.sum())
        for off in np.nonzero(eq)[0]:
            j = i + 1 + int(off)
            v = int(eq[off])
            if j - i < min_lag or flags[i] or flags[j]:
                continue
            e_voted += v
            n_distinct += 1
            if v >= min_votes:
                out.append((i, j, v))
    stats = dict(n_out=len(out), e_raw=e_raw, e_voted=e_voted, n_distinct=n_distinct,
                 n_flagged=int(flags.sum()), max_bucket=max_bucket)
    return out, stats, flags
