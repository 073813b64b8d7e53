"""GPU parity of the serving form: chunks searched against resident station
tables as they arrive.

The union of a station's chunk results must be exactly the oracle's search
of the concatenated station (history followed by the chunks) restricted to
pairs whose later member lies in a chunk, and the chunk counters must add up
to the oracle's counters of the concatenation minus those of the history.
Results must not depend on how chunks were batched (alone or mixed with
other stations' chunks) or on when the delta tables were merged.
"""
import sys

import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_1803_09835_amd as fl  # noqa: E402


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _fixed(n, dim, nnz, seed):
    rng = np.random.default_rng(seed)
    rows = [np.sort(rng.choice(dim, nnz, replace=False)) for _ in range(n)]
    return np.stack(rows).astype(np.uint16) if n else np.empty((0, nnz), np.uint16)


def _expected(rows, n_hist, dim, t, r, scheme, a, b, L, v):
    """Oracle pairs of the concatenation with j >= n_hist, and the counter
    differences (concatenation minus history)."""
    ei, ej, ev, est = oracle.search(rows, dim, t, r, scheme, a, b, L, v)
    keep = ej >= n_hist
    if n_hist:
        _, _, _, hst = oracle.search(rows[:n_hist], dim, t, r, scheme, a, b, L, v)
    else:
        hst = oracle.Stats(0, 0, 0, 0, 0, 0)
    diff = {k: getattr(est, k) - getattr(hst, k) for k in ("e_raw", "e_voted", "n_distinct")}
    return ei[keep], ej[keep], ev[keep], diff


def _run(stations, chunk_rows, dim, t, r, scheme, seed, L, v, order, **cfg):
    """stations: history arrays; chunk_rows[s]: list of chunk arrays of
    station s; order: (station, chunk index) submission order.  Returns
    per station the concatenated results and summed counters."""
    a, b = fl.make_hash(seed, fl.n_funcs(t, r, scheme))
    sv = fl.Server(dim, t, r, scheme, a, b, L, v, **cfg)
    ids = [sv.add_station(fl.to_device_rows(h)) for h in stations]
    dev = {(s, c): fl.to_device_rows(x) for s, xs in enumerate(chunk_rows) for c, x in enumerate(xs)}
    tickets = [(s, c, sv.submit(ids[s], dev[(s, c)])) for s, c in order]
    got = {s: {} for s in range(len(stations))}
    for s, c, tk in tickets:
        st, _ = sv.poll(tk, wait=True)
        oi, oj, ov = sv.take(tk)
        assert len(oi) == st.n_out
        got[s][c] = (oi, oj, ov, st)
    info = sv.info()
    sv.close()
    out = []
    for s in range(len(stations)):
        parts = [got[s][c] for c in sorted(got[s])]
        gi = np.concatenate([p[0] for p in parts]) if parts else np.empty(0, np.uint32)
        gj = np.concatenate([p[1] for p in parts]) if parts else np.empty(0, np.uint32)
        gv = np.concatenate([p[2] for p in parts]) if parts else np.empty(0, np.uint8)
        o = np.lexsort((gj, gi))
        sums = {k: sum(getattr(p[3], k) for p in parts) for k in ("e_raw", "e_voted", "n_distinct")}
        out.append((gi[o], gj[o], gv[o], sums, parts))
    return out, a, b, info


def _check(out, stations, chunk_rows, dim, t, r, scheme, a, b, L, v):
    for s, (gi, gj, gv, sums, _) in enumerate(out):
        rows = np.concatenate([stations[s]] + list(chunk_rows[s]))
        ei, ej, ev, diff = _expected(rows, len(stations[s]), dim, t, r, scheme, a, b, L, v)
        say(f"[serve] station {s}: {len(gi)} pairs (oracle {len(ei)}), counters {sums} vs {diff}")
        assert np.array_equal(gi, ei) and np.array_equal(gj, ej) and np.array_equal(gv, ev)
        assert sums == diff


def _chunks(rows, n_hist, sizes):
    out, p = [], n_hist
    for z in sizes:
        out.append(rows[p:p + z])
        p += z
    assert p == len(rows)
    return out


def test_serving_one_station_matches_batch_search():
    sizes = [3600] * 7 + [1000]
    n_hist = 25_000
    rows = synth.generate(synth.station(n=n_hist + sum(sizes), seed=160))
    hist, chunks = rows[:n_hist], _chunks(rows, n_hist, sizes)
    order = [(0, c) for c in range(len(chunks))]
    # a small delta forces several merges of the delta into the history
    out, a, b, info = _run([hist], [chunks], 4096, 100, 4, fl.MINMAX, 204, 5, 4, order, delta_rows=8000,
                           slack_rows=40_000)
    assert info["chunks"] == len(chunks)
    _check(out, [hist], [chunks], 4096, 100, 4, fl.MINMAX, a, b, 5, 4)
    assert len(out[0][0]) > 0


def test_serving_alone_and_mixed_batches_agree():
    # three stations (one with an empty history), chunks interleaved;
    # max_batch 1 runs every chunk alone, max_batch 8 mixes stations in a batch
    hists, chunk_rows = [], []
    for s, (nh, sizes) in enumerate([(15_000, [3600, 2000, 3600]), (8_000, [500, 3600, 3600, 77]),
                                     (0, [3600, 1200])]):
        rows = synth.generate(synth.station(n=nh + sum(sizes), seed=170 + s))
        hists.append(rows[:nh])
        chunk_rows.append(_chunks(rows, nh, sizes))
    order = []
    for c in range(4):
        for s in range(3):
            if c < len(chunk_rows[s]):
                order.append((s, c))
    runs = {}
    for mb in (1, 8):
        say(f"[serve] max_batch={mb}")
        runs[mb], a, b, info = _run(hists, chunk_rows, 4096, 100, 4, fl.MINMAX, 204, 5, 4, order, max_batch=mb,
                                    delta_rows=6000, slack_rows=20_000)
        if mb == 1:
            assert info["largest_batch"] == 1
        else:  # chunks of different stations did share a batch
            assert info["largest_batch"] > 1
        _check(runs[mb], hists, chunk_rows, 4096, 100, 4, fl.MINMAX, a, b, 5, 4)
    for s in range(3):  # per-chunk results identical, not only their union
        for p1, p8 in zip(runs[1][s][4], runs[8][s][4]):
            for x, y in zip(p1[:3], p8[:3]):
                assert np.array_equal(x, y)
            assert p1[3] == p8[3]


def test_serving_minhash_small_chunks_and_zero_lag():
    sizes = [1, 7, 4096, 300, 1]
    n_hist = 10_000
    rows = synth.generate(synth.tiny_uniform(n=n_hist + sum(sizes), seed=180))
    hist, chunks = rows[:n_hist], _chunks(rows, n_hist, sizes)
    for L, v in ((0, 1), (5, 2)):
        say(f"[serve] minhash L={L} v={v}")
        out, a, b, _ = _run([hist], [chunks], 4096, 20, 4, fl.MINHASH, 181, L, v,
                            [(0, c) for c in range(len(chunks))], max_chunk=4096, delta_rows=4096)
        _check(out, [hist], [chunks], 4096, 20, 4, fl.MINHASH, a, b, L, v)


def test_serving_huge_buckets_windowed():
    # identical rows: every query shares its bucket with every earlier row in
    # all tables, far more members than one counting pass holds
    base = _fixed(1, 4096, 200, 190)
    rows = np.concatenate([np.repeat(base, 6000, axis=0), _fixed(2000, 4096, 200, 191)])
    rng = np.random.default_rng(192)
    rows = rows[rng.permutation(len(rows))]
    n_hist = 5000
    sizes = [1000, 1000, 1000]
    hist, chunks = rows[:n_hist], _chunks(rows, n_hist, sizes)
    out, a, b, _ = _run([hist], [chunks], 4096, 12, 4, fl.MINMAX, 193, 3, 2, [(0, c) for c in range(3)],
                        max_chunk=1000, delta_rows=1500)
    _check(out, [hist], [chunks], 4096, 12, 4, fl.MINMAX, a, b, 3, 2)
    assert out[0][4][0][3].max_bucket > 4000


def test_serving_rejects_bad_chunk_and_keeps_station():
    sizes = [2000, 2000]
    n_hist = 6000
    rows = synth.generate(synth.station(n=n_hist + sum(sizes), seed=200))
    hist, chunks = rows[:n_hist], _chunks(rows, n_hist, sizes)
    a, b = fl.make_hash(201, 200)
    sv = fl.Server(4096, 100, 4, fl.MINMAX, a, b, 5, 4, max_chunk=4096)
    st = sv.add_station(fl.to_device_rows(hist))
    bad = chunks[0].copy()
    bad[17, 3] = 5000  # index >= dim
    tb = sv.submit(st, fl.to_device_rows(bad))
    with pytest.raises(fl.FastLshError) as e:
        sv.poll(tb, wait=True)
    assert e.value.code == 1
    d0, d1 = fl.to_device_rows(chunks[0]), fl.to_device_rows(chunks[1])
    t0, t1 = sv.submit(st, d0), sv.submit(st, d1)
    got = [sv.take(t0), sv.take(t1)]
    with pytest.raises(fl.FastLshError) as e:  # stations are added before serving starts
        sv.add_station(fl.to_device_rows(hist))
    assert e.value.code == 5
    sv.close()
    gi = np.concatenate([g[0] for g in got])
    gj = np.concatenate([g[1] for g in got])
    ei, ej, ev, _ = _expected(rows, n_hist, 4096, 100, 4, fl.MINMAX, a, b, 5, 4)
    o = np.lexsort((gj, gi))
    assert np.array_equal(gi[o], ei) and np.array_equal(gj[o], ej)


def test_serving_admission_and_arguments():
    a, b = fl.make_hash(1, 200)
    hist = fl.to_device_rows(_fixed(20_000, 4096, 200, 3))
    sv = fl.Server(4096, 100, 4, fl.MINMAX, a, b, 5, 4, hbm_budget=50 << 20)
    with pytest.raises(fl.FastLshError) as e:
        sv.add_station(hist)
    assert e.value.code == 2
    sv.close()
    with pytest.raises(fl.FastLshError):
        fl.Server(4096, 100, 4, fl.MINMAX, a, b, 5, 4, max_chunk=5000)
    sv = fl.Server(4096, 100, 4, fl.MINMAX, a, b, 5, 4)
    st = sv.add_station(hist)
    with pytest.raises(fl.FastLshError):
        sv.submit(st, fl.to_device_rows(_fixed(3601, 4096, 200, 4)))
    with pytest.raises(fl.FastLshError):
        sv.submit(st + 1, fl.to_device_rows(_fixed(10, 4096, 200, 4)))
    sv.close()


def test_serving_admits_chunks_by_station_room():
    # history 6,000 rows with room for 5,000 more, delta 4,000: chunks
    # already queued count against the room, a chunk that does not fit is
    # refused at submit (E_NOMEM) and leaves the station as it was, a chunk
    # that fails (a bad row) gives its rows back, and the admitted chunks'
    # results are exact (the third one's insertion merges the full delta
    # into the history)
    n_hist = 6000
    rows = synth.generate(synth.station(n=n_hist + 7000, seed=210))
    a, b = fl.make_hash(211, 200)
    sv = fl.Server(4096, 100, 4, fl.MINMAX, a, b, 5, 4, max_chunk=2000, delta_rows=4000, slack_rows=5000)
    st = sv.add_station(fl.to_device_rows(rows[:n_hist]))
    dev = lambda x: fl.to_device_rows(np.ascontiguousarray(x))  # noqa: E731
    t0 = sv.submit(st, dev(rows[6000:8000]))
    t1 = sv.submit(st, dev(rows[8000:10000]))
    with pytest.raises(fl.FastLshError) as e:  # 10,000 + 2,000 rows > 11,000
        sv.submit(st, dev(rows[10000:12000]))
    assert e.value.code == 2
    bad = rows[10000:11000].copy()
    bad[17, -1] = 5000  # an index >= dim: the chunk fails on the device
    tb = sv.submit(st, dev(bad))
    with pytest.raises(fl.FastLshError) as e:  # the bad chunk still holds its rows
        sv.submit(st, dev(rows[11000:11001]))
    assert e.value.code == 2
    with pytest.raises(fl.FastLshError) as e:
        sv.poll(tb, wait=True)
    assert e.value.code == 1
    t2 = sv.submit(st, dev(rows[10000:11000]))
    got = [sv.take(tk) for tk in (t0, t1, t2)]
    with pytest.raises(fl.FastLshError) as e:  # the station is full now
        sv.submit(st, dev(rows[11000:11001]))
    assert e.value.code == 2
    sv.close()
    ei, ej, ev, _ = _expected(rows[:11000], n_hist, 4096, 100, 4, fl.MINMAX, a, b, 5, 4)
    gi = np.concatenate([g[0] for g in got])
    gj = np.concatenate([g[1] for g in got])
    gv = np.concatenate([g[2] for g in got])
    o = np.lexsort((gj, gi))
    say(f"[serve] admission by room: {len(gi)} pairs (oracle {len(ei)})")
    assert np.array_equal(gi[o], ei) and np.array_equal(gj[o], ej) and np.array_equal(gv[o], ev)


def test_serving_small_station_merges_before_large_one():
    # Station 1 (4,000 history rows) fills its delta and merges into its
    # history before station 0 (20,000 rows) does.  The shared merge buffer
    # must still hold the larger station afterwards, and every chunk of both
    # stations must match the oracle.
    sizes = {0: [2000] * 5, 1: [2000] * 5}
    hist_n = {0: 20_000, 1: 4_000}
    rows = {s: synth.generate(synth.station(n=hist_n[s] + sum(sizes[s]), seed=220 + s)) for s in (0, 1)}
    hists = [rows[s][:hist_n[s]] for s in (0, 1)]
    chunk_rows = [_chunks(rows[s], hist_n[s], sizes[s]) for s in (0, 1)]
    a, b = fl.make_hash(221, 200)
    sv = fl.Server(4096, 100, 4, fl.MINMAX, a, b, 5, 4, max_batch=4, max_chunk=2000, delta_rows=4000,
                   slack_rows=12_000)
    ids = [sv.add_station(fl.to_device_rows(h)) for h in hists]
    dev = {(s, c): fl.to_device_rows(x) for s in (0, 1) for c, x in enumerate(chunk_rows[s])}
    got = {0: {}, 1: {}}

    def run(order):
        tks = [(s, c, sv.submit(ids[s], dev[(s, c)])) for s, c in order]
        for s, c, tk in tks:
            st, _ = sv.poll(tk, wait=True)
            got[s][c] = (*sv.take(tk), st)

    # the small station's third chunk finds its delta full: its merge runs
    # (after that batch) before any chunk of the large station is submitted
    run([(1, 0), (1, 1), (1, 2)])
    say("[serve] small station merged")
    run([(0, 0), (0, 1), (0, 2)])  # the large station's merge
    say("[serve] large station merged")
    run([(1, 3), (0, 3), (1, 4), (0, 4)])
    sv.close()
    out = []
    for s in (0, 1):
        parts = [got[s][c] for c in sorted(got[s])]
        gi = np.concatenate([p[0] for p in parts])
        gj = np.concatenate([p[1] for p in parts])
        gv = np.concatenate([p[2] for p in parts])
        o = np.lexsort((gj, gi))
        sums = {k: sum(getattr(p[3], k) for p in parts) for k in ("e_raw", "e_voted", "n_distinct")}
        out.append((gi[o], gj[o], gv[o], sums, parts))
    _check(out, hists, chunk_rows, 4096, 100, 4, fl.MINMAX, a, b, 5, 4)
