"""Pins of the oracle's section 6.4 / 6.5 forms: query-only hashing against
the direct vote definition and against the whole search of dataset plus
queries; the partitioned search with the dynamic occurrence filter against a
step-by-step brute force on a dense vote matrix, and (filter off) against
the whole search."""
import numpy as np
import pytest

import oracle
import synth
from brute import partitioned_brute, query_brute

DIM = 4096


def _keys(rows, t, r, scheme, seed):
    a, b = oracle.make_hash(seed, oracle.n_funcs(t, r, scheme))
    return oracle.signatures(rows, DIM, t, r, scheme, a, b)


@pytest.mark.parametrize("v", [1, 2, 4])
def test_query_matches_direct_votes(v):
    rows = synth.generate(synth.station(n=3000, seed=5))
    keys = _keys(rows, 30, 4, oracle.MINMAX, 6)
    qsel = np.r_[10:40, 1500:1530, 2990:3000]  # queries: copies of some rows plus their neighbours
    q, x, vv, nc = oracle.query_keys(keys[:, qsel], keys, v)
    wq, wx, wv = query_brute(keys[:, qsel], keys, v)
    assert np.array_equal(q, wq) and np.array_equal(x, wx) and np.array_equal(vv, wv)
    # every query finds itself in every table
    self_hits = vv[x == qsel[q]]
    assert len(self_hits) == len(qsel) and (self_hits == 30).all()
    assert nc >= int(wv.astype(np.int64).sum())


def test_query_equals_whole_search_of_dataset_and_queries():
    # section 6.4: hashing only the queries gives the whole search's results
    d = synth.generate(synth.station(n=2000, seed=7))
    qrows = synth.generate(synth.Spec(n=300, seed=8))
    qrows[:50] = d[100:150]  # some queries repeat dataset rows
    both = np.concatenate([d, qrows])
    keys = _keys(both, 20, 4, oracle.MINHASH, 9)
    i, j, v, _ = oracle.search_keys(keys, 1, 2)
    cross = (i < len(d)) & (j >= len(d))
    want = sorted(zip((j[cross] - len(d)).tolist(), i[cross].tolist(), v[cross].tolist()))
    q, x, vv, _ = oracle.query_keys(keys[:, len(d):], keys[:, :len(d)], 2)
    assert list(zip(q.tolist(), x.tolist(), vv.tolist())) == want and len(want) > 50


@pytest.mark.parametrize("parts", [1, 2, 3, 7])
def test_partitioned_without_filter_is_the_whole_search(parts):
    rows = synth.generate(synth.station(n=4000, seed=11))
    keys = _keys(rows, 40, 4, oracle.MINMAX, 12)
    whole = oracle.search_keys(keys, 5, 3)
    got = oracle.search_partitioned_keys(keys, 5, 3, 0, 0, parts)
    for g, w in zip(got[:3], whole[:3]):
        assert np.array_equal(g, w)
    gs, ws = got[3].__dict__, whole[3].__dict__
    assert gs == ws


@pytest.mark.parametrize("parts,num,den,lag,v", [(1, 1, 10, 5, 2), (2, 1, 10, 5, 2), (3, 1, 20, 2, 1),
                                                 (4, 1, 50, 5, 3), (5, 3, 100, 0, 2)])
def test_partitioned_filter_matches_brute_force(parts, num, den, lag, v):
    # repeating noise (near-copies of one template) in a short station
    rows = synth.generate(synth.with_noise(synth.station(n=500, seed=13 + parts), 120, 190))
    keys = _keys(rows, 16, 4, oracle.MINMAX, 14)
    gi, gj, gv, gst, ex = oracle.search_partitioned_keys(keys, lag, v, num, den, parts, want_excluded=True)
    wi, wj, wv, wst = partitioned_brute(keys, lag, v, num, den, parts)
    assert np.array_equal(gi, wi) and np.array_equal(gj, wj) and np.array_equal(gv, wv)
    assert gst.__dict__ == wst
    assert gst.n_flagged > 0 and int(ex.sum()) == gst.n_flagged


def test_partition_threshold_uses_the_partition_size():
    # a burst of 80 identical rows in the second half: each has about 75
    # candidates, over 5 % of a 1000-row partition (50) but not of the whole
    # 2000-row station (100)
    rows = synth.generate(synth.station(n=2000, seed=21))
    rows[1500:1580] = rows[1500]
    keys = _keys(rows, 20, 4, oracle.MINMAX, 22)
    one = oracle.search_partitioned_keys(keys, 5, 2, 5, 100, 1, want_excluded=True)
    two = oracle.search_partitioned_keys(keys, 5, 2, 5, 100, 2, want_excluded=True)
    assert not one[4][1500:1580].any()
    assert two[4][1500:1580].all()
    assert not ((two[0] >= 1500) & (two[0] < 1580)).any() and ((one[0] >= 1500) & (one[0] < 1580)).any()
