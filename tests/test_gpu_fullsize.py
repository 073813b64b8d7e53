"""GPU parity at the full workload sizes, on samples the oracle can check
one by one.

The 90-day station (7,776,000 fingerprints) with the search bench.py times,
and the 5-year station (157,788,000 fingerprints) with the bounded-memory
search, in the same launch configuration.  The oracle cannot search these
sizes whole, so it checks, exactly:
  - every reported pair is canonical (i < j, sorted, lag and threshold kept);
  - sampled reported pairs carry exactly the oracle's vote count;
  - completeness on samples: pairs of copies of one planted source, and
    pairs at short lags, that reach the threshold in the oracle are reported;
  - the occurrence filter cannot fire here (largest bucket below 1 % of n),
    and no fingerprint is excluded.
"""
import hashlib
import json
import os
import sys
import time

import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_1803_09835_amd as fl  # noqa: E402

DIM, T, R, SCHEME, L, V, NUM, DEN = 4096, 100, 4, fl.MINMAX, 5, 4, 1, 100


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _upload(spec, chunk=16_000_000):
    """Rows to the device chunk by chunk through a pinned buffer; labels on the host."""
    dev = torch.empty((spec.n, spec.nnz), dtype=torch.int16, device="cuda")
    labels = np.empty(spec.n, dtype=np.int32)
    pinned = torch.empty((min(chunk, spec.n), spec.nnz), dtype=torch.int16, pin_memory=True)
    for lo in range(0, spec.n, chunk):
        hi = min(spec.n, lo + chunk)
        _, lab = synth.generate(spec, lo, hi, labels=True, out=pinned[: hi - lo].numpy().view(np.uint16))
        labels[lo:hi] = lab
        dev[lo:hi].copy_(pinned[: hi - lo])
        say(f"[upload] rows {lo}..{hi}")
    return dev, labels


def _oracle_votes(dev, a, b, pi, pj):
    ids = np.unique(np.concatenate([pi, pj]))
    rows = dev[torch.from_numpy(ids.astype(np.int64)).cuda()].cpu().numpy().view(np.uint16)
    keys = oracle.signatures(rows, DIM, T, R, oracle.MINMAX, a, b)
    x, y = np.searchsorted(ids, pi), np.searchsorted(ids, pj)
    return (keys[:, x] == keys[:, y]).sum(axis=0)


def _check_sampled(dev, labels, out, n, a, b, seed):
    gi, gj = out[0].cpu().numpy().view(np.uint32), out[1].cpu().numpy().view(np.uint32)
    gv, st = out[2].cpu().numpy(), out[3]
    say(f"[check] n={n} pairs={len(gi)} stats={st}")
    assert len(gi) == st.n_out > 0
    assert (gi < gj).all() and (gj - gi >= L).all() and (gv >= V).all() and (gv <= T).all()
    key = (gi.astype(np.uint64) << np.uint64(32)) | gj.astype(np.uint64)
    assert (key[1:] > key[:-1]).all()
    assert st.max_bucket * DEN <= n * NUM and st.n_flagged == 0
    assert st.e_voted >= gv.astype(np.int64).sum() and st.e_raw >= st.n_out
    rng = np.random.default_rng(seed)
    # reported pairs: exact votes
    k = rng.choice(len(gi), min(3000, len(gi)), replace=False)
    votes = _oracle_votes(dev, a, b, gi[k].astype(np.int64), gj[k].astype(np.int64))
    assert np.array_equal(votes, gv[k].astype(votes.dtype))
    # completeness: copies of planted sources, and short-lag pairs
    planted = np.flatnonzero(labels >= 0)
    srcs = rng.choice(np.unique(labels[planted]), 300, replace=False)
    pi, pj = [], []
    order = planted[np.argsort(labels[planted], kind="stable")]
    lab_sorted = labels[order]
    for s in srcs:
        members = np.sort(order[np.searchsorted(lab_sorted, s):np.searchsorted(lab_sorted, s, side="right")])
        for x in range(len(members)):
            for y in range(x + 1, len(members)):
                pi.append(members[x])
                pj.append(members[y])
    base = rng.integers(0, n - 64, 2000)
    lag = rng.integers(L, 64, 2000)
    pi = np.concatenate([np.array(pi, dtype=np.int64), base])
    pj = np.concatenate([np.array(pj, dtype=np.int64), base + lag])
    keep = pj - pi >= L
    pi, pj = pi[keep], pj[keep]
    votes = _oracle_votes(dev, a, b, pi, pj)
    want = votes >= V
    q = (pi.astype(np.uint64) << np.uint64(32)) | pj.astype(np.uint64)
    pos = np.searchsorted(key, q)
    found = (pos < len(key)) & (key[np.minimum(pos, len(key) - 1)] == q)
    say(f"[check] completeness sample {len(q)} pairs, {int(want.sum())} at or above the threshold")
    assert want.sum() > 50
    assert np.array_equal(found, want)
    got_v = gv[np.minimum(pos, len(key) - 1)][found]
    assert np.array_equal(got_v.astype(votes.dtype), votes[found])


GOLDEN_90D = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "station90d.json")
PAIR = np.dtype([("i", "<u4"), ("j", "<u4"), ("v", "u1")])


def _digest(out):
    rec = np.empty(len(out[0]), dtype=PAIR)
    rec["i"] = out[0].cpu().numpy().view(np.uint32)
    rec["j"] = out[1].cpu().numpy().view(np.uint32)
    rec["v"] = out[2].cpu().numpy()
    return hashlib.sha256(rec.tobytes()).hexdigest(), np.bincount(rec["v"], minlength=T + 1)


def test_station_90d_full_size():
    """The 90-day station searched as bench.py's station workload searches it,
    against the oracle's complete result (tests/golden/station90d.json, written
    by make_station90d.py from the oracle alone): the SHA-256 of the sorted
    output and every counter, with and without the distinct-pair count (the
    two take different row layouts), plus the sampled checks."""
    spec = synth.station(n=synth.STATION_90D, seed=102)
    say("[fullsize] station 90 days: generating")
    dev, labels = _upload(spec)
    a, b = fl.make_hash(202, fl.n_funcs(T, R, SCHEME))
    ctx = fl.FastLSH(0)
    gold = json.load(open(GOLDEN_90D))
    assert gold["n"] == spec.n and gold["data_seed"] == 102 and gold["hash_seed"] == 202
    for distinct in (False, True):
        t0 = time.time()
        out = ctx.search(dev, DIM, T, R, SCHEME, a, b, L, V, NUM, DEN, want_distinct=distinct)
        torch.cuda.synchronize()
        say(f"[fullsize] search (distinct={distinct}) {time.time() - t0:.2f}s: {out[3]}")
        dig, hist = _digest(out)
        got = dict(out[3].__dict__)
        want = dict(gold["stats"])
        if not distinct:
            assert got.pop("n_distinct") == 2**64 - 1
            want.pop("n_distinct")
        assert got == want
        assert {str(k): int(c) for k, c in enumerate(hist) if c} == gold["pairs_by_votes"]
        assert dig == gold["sha256_pairs"]
    _check_sampled(dev, labels, out, spec.n, a, b, 1)
    ctx.close()


GOLDEN_5Y = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "station5y_counters.json")


def test_station_5y_bounded_full_size():
    """The 5-year station searched as bench.py's default workload searches it
    (bounded search, tables 10 at a time): its exact global counters e_raw,
    max_bucket and n_flagged against the oracle's (tests/golden/
    station5y_counters.json, written by make_station5y_counters.py from the
    oracle alone, a few tables at a time), plus the sampled checks of the
    pairs."""
    gold = json.load(open(GOLDEN_5Y))
    spec = synth.long_station(n=synth.STATION_5Y, seed=105)
    assert gold["n"] == spec.n and gold["data_seed"] == 105 and gold["hash_seed"] == 205
    assert (gold["tables"], gold["rows"], gold["occ_num"], gold["occ_den"]) == (T, R, NUM, DEN)
    say("[fullsize] station 5 years: generating")
    dev, labels = _upload(spec)
    a, b = fl.make_hash(205, fl.n_funcs(T, R, SCHEME))
    ctx = fl.FastLSH(0)
    t0 = time.time()
    out = ctx.search_bounded(dev, DIM, T, R, SCHEME, a, b, L, V, NUM, DEN, group_tables=10)
    torch.cuda.synchronize()
    st = out[3]
    say(f"[fullsize] bounded search {time.time() - t0:.2f}s: {st}, groupings kept {ctx.config_used()['keep_groups']}")
    assert {"e_raw": st.e_raw, "max_bucket": st.max_bucket, "n_flagged": st.n_flagged} == gold["counters"]
    _check_sampled(dev, labels, out, spec.n, a, b, 2)
    ctx.close()


def test_serving_180d_full_size():
    """The serving workload at its full size: 8 stations with 180-day
    histories (15,552,000 fingerprints each, the recipe bench.py serves)
    resident, and 12 chunks of 3,600 fingerprints per station offered at
    once, so that batches mix stations.  Every chunk's pairs have their later
    member in the chunk, lie at or above the lag and the threshold and come
    sorted; sampled reported pairs carry exactly the oracle's votes; and
    every pair of copies of a planted source, and sampled short-lag pairs,
    whose later member lies in a chunk is reported exactly when the oracle's
    votes reach the threshold."""
    S, CH, NCH = 8, synth.CHUNK, 12
    n_hist = synth.STATION_180D
    n = n_hist + NCH * CH
    a, b = fl.make_hash(204, fl.n_funcs(T, R, SCHEME))
    sv = fl.Server(DIM, T, R, SCHEME, a, b, L, V, max_batch=8, max_chunk=CH, delta_rows=262144,
                   slack_rows=NCH * CH)
    host, labs, streams = [], [], []
    for s in range(S):
        spec = synth.Spec(n=n, seed=1040 + s, markov_keep=140, n_sources=4000, rep_min=3, rep_max=40,
                          jac_lo_milli=400, jac_hi_milli=900, chain_len=1_000_000)
        rows = np.empty((n, spec.nnz), dtype=np.uint16)
        _, lab = synth.generate(spec, 0, n, labels=True, out=rows)
        hist = torch.from_numpy(rows[:n_hist].view(np.int16)).cuda()
        assert sv.add_station(hist) == s
        del hist
        torch.cuda.empty_cache()
        streams.append(torch.from_numpy(rows[n_hist:].view(np.int16)).cuda())
        host.append(rows)
        labs.append(lab)
        say(f"[serve-full] station {s}: {n_hist} rows resident")
    tickets = {(s, c): sv.submit(s, streams[s][c * CH:(c + 1) * CH]) for c in range(NCH) for s in range(S)}
    got = {k: sv.take(tk) for k, tk in tickets.items()}
    info = sv.info()
    sv.close()
    say(f"[serve-full] {len(got)} chunks done, server {info}")
    assert info["largest_batch"] > 1
    rng = np.random.default_rng(7)
    total_want = 0
    for s in range(S):
        parts = []
        for c in range(NCH):
            oi, oj, ov = (x.astype(np.int64) for x in got[(s, c)])
            lo = n_hist + c * CH
            assert ((oj >= lo) & (oj < lo + CH)).all() and (oi < oj).all() and (oj - oi >= L).all()
            assert (ov >= V).all() and (ov <= T).all()
            key = (oi << 32) | oj
            assert (key[1:] > key[:-1]).all()
            parts.append((oi, oj, ov))
        gi = np.concatenate([p[0] for p in parts])
        gj = np.concatenate([p[1] for p in parts])
        gv = np.concatenate([p[2] for p in parts])
        key = (gi << 32) | gj
        o = np.argsort(key)
        key, gv = key[o], gv[o]
        rows, lab = host[s], labs[s]
        # reported pairs: exact votes
        k = rng.choice(len(key), min(400, len(key)), replace=False)
        votes = _host_votes(rows, a, b, key[k] >> 32, key[k] & 0xFFFFFFFF)
        assert np.array_equal(votes, gv[k])
        # completeness: every copy pair with its later copy in a chunk, and
        # short-lag pairs ending in the chunks
        planted = np.flatnonzero(lab >= 0)
        order = planted[np.argsort(lab[planted], kind="stable")]
        lab_sorted = lab[order]
        pi, pj = [], []
        for j in planted[planted >= n_hist]:
            members = order[np.searchsorted(lab_sorted, lab[j]):np.searchsorted(lab_sorted, lab[j], side="right")]
            for i in members[(members < j) & (j - members >= L)]:
                pi.append(i)
                pj.append(j)
        jj = rng.integers(n_hist, n, 500)
        ll = rng.integers(L, 64, 500)
        pi = np.concatenate([np.array(pi, dtype=np.int64), jj - ll])
        pj = np.concatenate([np.array(pj, dtype=np.int64), jj])
        votes = _host_votes(rows, a, b, pi, pj)
        want = votes >= V
        q = (pi << 32) | pj
        pos = np.minimum(np.searchsorted(key, q), len(key) - 1)
        found = key[pos] == q
        say(f"[serve-full] station {s}: {len(key)} pairs in its chunks; completeness sample {len(q)} pairs, "
            f"{int(want.sum())} at or above the threshold")
        assert np.array_equal(found, want)
        assert np.array_equal(gv[pos][found], votes[found])
        total_want += int(want.sum())
    assert total_want > 100


def _host_votes(rows, a, b, pi, pj):
    """Oracle votes of pairs (pi, pj) of host rows."""
    pi, pj = np.asarray(pi, dtype=np.int64), np.asarray(pj, dtype=np.int64)
    ids = np.unique(np.concatenate([pi, pj]))
    keys = oracle.signatures(np.ascontiguousarray(rows[ids]), DIM, T, R, oracle.MINMAX, a, b)
    x, y = np.searchsorted(ids, pi), np.searchsorted(ids, pj)
    return (keys[:, x] == keys[:, y]).sum(axis=0).astype(np.int64)


def test_batched_12_stations_full_size():
    """The batched workload at its full size (12 stations of 1-8, 10, 12, 14
    and 16 M uniform fingerprints with 50 x 5 planted copies each, 88 M in
    all; MinHash t=20 r=4, lag 5, v=2): the one batched search equals every
    station searched alone, element by element and counter by counter;
    sampled reported pairs carry the oracle's votes, and every pair of
    copies of a planted source is reported exactly when the oracle's votes
    reach the threshold."""
    t, r, scheme, lag, v = 20, 4, fl.MINHASH, 5, 2
    a, b = fl.make_hash(201, fl.n_funcs(t, r, scheme))
    hosts, labs, devs = [], [], []
    for s, m in enumerate(synth.BATCH_LENGTHS_M):
        spec = synth.tiny_uniform(n=m * 1_000_000, seed=1030 + s)
        rows = np.empty((spec.n, spec.nnz), dtype=np.uint16)
        _, lab = synth.generate(spec, 0, spec.n, labels=True, out=rows)
        hosts.append(rows)
        labs.append(lab)
        devs.append(torch.from_numpy(rows.view(np.int16)).cuda())
    say(f"[batched-full] {sum(len(x) for x in hosts)} fingerprints in {len(hosts)} stations")
    ctx = fl.FastLSH(0)
    bi, bj, bv, offs, bst = ctx.search_batched(devs, DIM, t, r, scheme, a, b, lag, v)
    torch.cuda.synchronize()
    rng = np.random.default_rng(12)
    total_want = 0
    for s, rows in enumerate(hosts):
        oi, oj, ov, st = ctx.search(devs[s], DIM, t, r, scheme, a, b, lag, v)
        lo, hi = int(offs[s]), int(offs[s + 1])
        assert torch.equal(bi[lo:hi], oi) and torch.equal(bj[lo:hi], oj) and torch.equal(bv[lo:hi], ov)
        assert bst[s] == st
        gi = oi.cpu().numpy().view(np.uint32).astype(np.int64)
        gj = oj.cpu().numpy().view(np.uint32).astype(np.int64)
        gv = ov.cpu().numpy().astype(np.int64)
        key = (gi << 32) | gj
        k = rng.choice(len(key), min(300, len(key)), replace=False)
        assert np.array_equal(_minhash_votes(rows, a, b, t, r, gi[k], gj[k]), gv[k])
        lab = labs[s]
        planted = np.flatnonzero(lab >= 0)
        pi, pj = [], []
        for src in np.unique(lab[planted]):
            members = np.sort(planted[lab[planted] == src])
            for x in range(len(members)):
                for y in range(x + 1, len(members)):
                    if members[y] - members[x] >= lag:
                        pi.append(members[x])
                        pj.append(members[y])
        pi, pj = np.array(pi, dtype=np.int64), np.array(pj, dtype=np.int64)
        votes = _minhash_votes(rows, a, b, t, r, pi, pj)
        want = votes >= v
        q = (pi << 32) | pj
        pos = np.minimum(np.searchsorted(key, q), len(key) - 1)
        found = key[pos] == q
        say(f"[batched-full] station {s}: {hi - lo} pairs, {st}; planted pairs {len(q)}, {int(want.sum())} at or "
            f"above the threshold")
        assert np.array_equal(found, want)
        assert np.array_equal(gv[pos][found], votes[found])
        total_want += int(want.sum())
    assert total_want > 100
    ctx.close()


def _minhash_votes(rows, a, b, t, r, pi, pj):
    """Oracle votes (MinHash) of pairs (pi, pj) of host rows."""
    ids = np.unique(np.concatenate([pi, pj]))
    keys = oracle.signatures(np.ascontiguousarray(rows[ids]), DIM, t, r, oracle.MINHASH, a, b)
    x, y = np.searchsorted(ids, pi), np.searchsorted(ids, pj)
    return (keys[:, x] == keys[:, y]).sum(axis=0).astype(np.int64)
