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


def channel_merge_brute(channels, min_sim):
    """Combined similarity by a hash map of (dt, idx1) -> summed sim (the
    'naive' shared-map route section 7.2 describes), filtered and sorted."""
    acc = {}
    for i, j, v in channels:
        for x, y, s in zip(i.tolist(), j.tolist(), v.tolist()):
            assert y > x
            acc[(y - x, x)] = acc.get((y - x, x), 0) + s
    keys = sorted(k for k, s in acc.items() if s >= min_sim)
    return (np.array([k[0] for k in keys], dtype=np.uint32), np.array([k[1] for k in keys], dtype=np.uint32),
            np.array([acc[k] for k in keys], dtype=np.uint32))


def station_clusters_brute(dt, idx1, sim, max_gap, max_width, min_entries=1, min_sum=0):
    """Clusters as connected components of the entries themselves: two
    entries are neighbours when their diagonals differ by at most one and
    their start times by at most max_gap (O(E^2), no runs, no union-find).
    Returns a list of tuples in the field order of oracle.CLUSTER_DTYPE, in
    the order of each cluster's first entry."""
    n = len(dt)
    dt = [int(x) for x in dt]
    idx1 = [int(x) for x in idx1]
    sim = [int(x) for x in sim]
    comp = [-1] * n
    for s in range(n):
        if comp[s] >= 0:
            continue
        comp[s] = s
        stack = [s]
        while stack:
            a = stack.pop()
            for b in range(n):
                if comp[b] < 0 and abs(dt[a] - dt[b]) <= 1 and abs(idx1[a] - idx1[b]) <= max_gap:
                    comp[b] = s
                    stack.append(b)
    out = []
    for c in sorted(set(comp)):  # the first entry of each component, in input order
        mem = [k for k in range(n) if comp[k] == c]
        d = [dt[k] for k in mem]
        x = [idx1[k] for k in mem]
        peak = min(mem, key=lambda k: (-sim[k], dt[k], idx1[k]))
        tot = sum(sim[k] for k in mem)
        if max(d) - min(d) + 1 > max_width or len(mem) < min_entries or tot < min_sum:
            continue
        out.append((min(d), max(d), min(x), max(x), len(mem), sim[peak], dt[peak], idx1[peak], tot))
    return out


def vote_matrix(keys):
    """votes[i, j] = number of tables whose keys of i and j are equal (dense)."""
    t, n = keys.shape
    v = np.zeros((n, n), dtype=np.int64)
    for u in range(t):
        v += keys[u][:, None] == keys[u][None, :]
    return v


def query_brute(qkeys, dkeys, min_votes):
    """Query-only result straight from the definition: votes[q, x] counted by
    comparing every query's keys with every item's keys."""
    v = np.zeros((qkeys.shape[1], dkeys.shape[1]), dtype=np.int64)
    for u in range(qkeys.shape[0]):
        v += qkeys[u][:, None] == dkeys[u][None, :]
    q, x = np.nonzero(v >= min_votes)
    return q.astype(np.uint32), x.astype(np.uint32), v[q, x].astype(np.uint8)


def partitioned_brute(keys, min_lag, min_votes, occ_num, occ_den, n_parts):
    """The partitioned search with the dynamic occurrence filter, step by step
    on a dense vote matrix (no buckets).  Returns (i, j, votes, counters)."""
    t, n = keys.shape
    v = vote_matrix(keys)
    ex = np.zeros(n, dtype=bool)
    idx = np.arange(n)
    out, e_voted, n_distinct = [], 0, 0
    for p in range(n_parts):
        lo, hi = n * p // n_parts, n * (p + 1) // n_parts
        cands = {}
        for i in range(lo, hi):
            if ex[i]:
                continue
            ok = (v[i] >= 1) & (idx != i) & (np.abs(idx - i) >= min_lag) & ~ex
            cands[i] = np.flatnonzero(ok)
        if occ_den:
            newly = set()
            for i, c in cands.items():
                if len(c) * occ_den > (hi - lo) * occ_num:
                    newly.add(i)
                    newly.update(int(j) for j in c)
            ex[list(newly)] = True
        for i in range(lo, hi):
            if ex[i]:
                continue
            for j in range(i + min_lag if min_lag > 0 else i + 1, n):
                if j <= i or ex[j] or v[i, j] == 0:
                    continue
                e_voted += int(v[i, j])
                n_distinct += 1
                if v[i, j] >= min_votes:
                    out.append((i, j, int(v[i, j])))
    iu = np.triu_indices(n, 1)
    e_raw = int(v[iu].sum())
    max_bucket = max(int(np.unique(keys[u], return_counts=True)[1].max()) for u in range(t)) if n else 0
    st = dict(n_out=len(out), e_raw=e_raw, e_voted=e_voted, n_distinct=n_distinct, n_flagged=int(ex.sum()),
              max_bucket=max_bucket)
    return (np.array([o[0] for o in out], np.uint32), np.array([o[1] for o in out], np.uint32),
            np.array([o[2] for o in out], np.uint8), st)
