"""Pins of the oracle's spatiotemporal alignment (section 7): the channel
merge against a hash-map brute force and hand-worked cases; the station
clusters against a component search over the entries themselves (no runs,
no union-find) and hand-worked boundary cases."""
import numpy as np
import pytest

import oracle
from align_inputs import channels as _channels, entries as _entries
from brute import channel_merge_brute, station_clusters_brute


@pytest.mark.parametrize("seed,min_sim", [(1, 0), (2, 1), (3, 8), (4, 20), (5, 40)])
def test_channel_merge_matches_hash_map(seed, min_sim):
    ch = _channels(seed)
    got = oracle.channel_merge(ch, min_sim)
    want = channel_merge_brute(ch, min_sim)
    for g, w in zip(got, want):
        assert np.array_equal(g, w)


def test_channel_merge_hand_worked():
    # channel 0: (i, j, v) = (1, 5, 3), (2, 3, 1); channel 1: (1, 5, 2), (0, 4, 4)
    # -> (dt, idx1) keys: (4, 1): 3 + 2 = 5; (1, 2): 1; (4, 0): 4.
    c0 = (np.array([1, 2], np.uint32), np.array([5, 3], np.uint32), np.array([3, 1], np.uint8))
    c1 = (np.array([0, 1], np.uint32), np.array([4, 5], np.uint32), np.array([4, 2], np.uint8))
    dt, idx1, sim = oracle.channel_merge([c0, c1], 0)
    assert dt.tolist() == [1, 4, 4] and idx1.tolist() == [2, 0, 1] and sim.tolist() == [1, 4, 5]
    dt, idx1, sim = oracle.channel_merge([c0, c1], 5)
    assert dt.tolist() == [4] and idx1.tolist() == [1] and sim.tolist() == [5]


def test_channel_merge_invariants():
    ch = _channels(9, n_ch=4)
    # one channel: its own triplets, re-ordered by (dt, idx1)
    i, j, v = ch[0]
    dt, idx1, sim = oracle.channel_merge([ch[0]], 0)
    order = np.lexsort((i, j - i))
    assert np.array_equal(dt, (j - i)[order]) and np.array_equal(idx1, i[order]) and np.array_equal(sim, v[order])
    # nothing is lost without a threshold, and the channel order does not matter
    dt, idx1, sim = oracle.channel_merge(ch, 0)
    assert int(sim.sum()) == sum(int(c[2].sum()) for c in ch)
    assert len(dt) == len({(int(b) - int(a), int(a)) for c in ch for a, b in zip(c[0], c[1])})
    rev = oracle.channel_merge(ch[::-1], 0)
    assert all(np.array_equal(x, y) for x, y in zip((dt, idx1, sim), rev))
    assert [len(x) for x in oracle.channel_merge([], 0)] == [0, 0, 0]
    with pytest.raises(ValueError):
        oracle.channel_merge([(np.array([3], np.uint32), np.array([3], np.uint32), np.array([1], np.uint8))], 0)


@pytest.mark.parametrize("seed,gap,width,me,ms", [(1, 1, 1, 1, 0), (2, 3, 2, 2, 0), (3, 5, 3, 3, 20),
                                                  (4, 10, 12, 1, 0), (5, 0, 5, 1, 0), (6, 4, 1, 5, 40)])
def test_station_clusters_match_component_search(seed, gap, width, me, ms):
    dt, idx1, sim = _entries(seed)
    got = oracle.station_clusters(dt, idx1, sim, gap, width, me, ms)
    want = station_clusters_brute(dt, idx1, sim, gap, width, me, ms)
    assert [tuple(int(x) for x in row) for row in got] == want


def test_station_clusters_hand_worked():
    # diagonal 10: idx1 0, 2, 4 (gaps 2) and 9 (gap 5); diagonal 11: idx1 6, 7;
    # diagonal 13: idx1 3.
    dt = np.array([10, 10, 10, 10, 11, 11, 13], np.uint32)
    idx1 = np.array([0, 2, 4, 9, 6, 7, 3], np.uint32)
    sim = np.array([5, 7, 7, 2, 1, 9, 4], np.uint32)
    # gap 2: runs {0,2,4}, {9}, {6,7} (dt 11), {3} (dt 13); {6,7} is within 2
    # of both {0..4} (6 <= 4 + 2) and {9} (9 <= 7 + 2), so three runs join;
    # dt 13 is two diagonals away and stays alone.
    c = oracle.station_clusters(dt, idx1, sim, 2, 2)
    rows = [tuple(int(x) for x in r) for r in c]
    assert rows == [(10, 11, 0, 9, 6, 9, 11, 7, 31), (13, 13, 3, 3, 1, 4, 13, 3, 4)]
    # gap 1: diagonal 10 splits into four single-entry runs, {6, 7} stays one
    # run, and no run of diagonal 10 comes within 1 of it (4 -> 6 is 2,
    # 7 -> 9 is 2): six clusters
    c = oracle.station_clusters(dt, idx1, sim, 1, 5)
    assert len(c) == 6
    # width 1 prunes the two-diagonal cluster; min_entries 2 prunes singletons
    c = oracle.station_clusters(dt, idx1, sim, 2, 1)
    assert [int(r["dt_min"]) for r in c] == [13]
    c = oracle.station_clusters(dt, idx1, sim, 2, 2, 2)
    assert [int(r["n_entries"]) for r in c] == [6]
    # peak ties go to the earlier entry: sims 7 at (10, 2) and (10, 4)
    c = oracle.station_clusters(dt[:3], idx1[:3], sim[:3], 2, 1)
    assert (int(c[0]["peak_dt"]), int(c[0]["peak_idx1"]), int(c[0]["peak_sim"])) == (10, 2, 7)
    with pytest.raises(ValueError):
        oracle.station_clusters(dt[::-1].copy(), idx1[::-1].copy(), sim, 2, 2)


def test_station_clusters_partition_every_entry():
    dt, idx1, sim = _entries(11, noise=300)
    c = oracle.station_clusters(dt, idx1, sim, 3, 10**6)
    assert int(c["n_entries"].sum()) == len(dt) and int(c["sim_sum"].sum()) == int(sim.sum())
    assert len(oracle.station_clusters(dt[:0], idx1[:0], sim[:0], 3, 3)) == 0
