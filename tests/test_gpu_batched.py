"""GPU parity of the batched (multi-station) search, graph replay and launch
shapes.

The batched search must give, for every station, exactly what the oracle
gives for that station alone (pairs, votes and counters, with the occurrence
filter using the station's own n); graph replays and every launch shape must
give the eager default's output bytes.
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


@pytest.fixture(scope="module")
def ctx():
    c = fl.FastLSH(0)
    yield c
    c.close()


def _np(t, dt):
    return t.cpu().numpy().view(dt)


def _fixed(n, dim, nnz, seed):
    rng = np.random.default_rng(seed)
    rows = [np.sort(rng.choice(dim, nnz, replace=False)) for _ in range(n)]
    return np.stack(rows).astype(np.uint16) if n else np.empty((0, nnz), np.uint16)


def _check_batched(ctx, stations, dim, t, r, scheme, seed, L, v, num=0, den=0, distinct=False, graph=False,
                   label=""):
    say(f"[batched] {label} sizes={[len(s) for s in stations]} t={t} r={r} scheme={scheme} L={L} v={v} "
        f"occ={num}/{den} distinct={distinct} graph={graph}")
    a, b = fl.make_hash(seed, fl.n_funcs(t, r, scheme))
    dev = [fl.to_device_rows(s) for s in stations]
    gi, gj, gv, offs, sts = ctx.search_batched(dev, dim, t, r, scheme, a, b, L, v, num, den,
                                               want_distinct=distinct, graph=graph)
    gi, gj, gv = _np(gi, np.uint32), _np(gj, np.uint32), gv.cpu().numpy()
    assert offs[0] == 0 and offs[-1] == len(gi) and (np.diff(offs) >= 0).all()
    for s, rows in enumerate(stations):
        lo, hi = offs[s], offs[s + 1]
        if len(rows) == 0:
            assert lo == hi and sts[s].e_raw == 0 and sts[s].n_out == 0
            continue
        ei, ej, ev, est = oracle.search(rows, dim, t, r, scheme, a, b, L, v, num, den)
        assert hi - lo == len(ei), (s, hi - lo, len(ei))
        assert np.array_equal(gi[lo:hi], ei), s
        assert np.array_equal(gj[lo:hi], ej), s
        assert np.array_equal(gv[lo:hi], ev), s
        want, got = dict(est.__dict__), dict(sts[s].__dict__)
        if not distinct:
            assert got.pop("n_distinct") == 2**64 - 1
            want.pop("n_distinct")
        assert got == want, (s, got, want)
    return (gi, gj, gv, offs, sts)


def test_batched_uniform_stations(ctx):
    sizes = (20_000, 7_000, 0, 13_000, 1, 9_000)
    stations = [synth.generate(synth.tiny_uniform(n=n, seed=1030 + s)) if n > 1000 else _fixed(n, 4096, 200, s)
                for s, n in enumerate(sizes)]
    out = _check_batched(ctx, stations, 4096, 20, 4, fl.MINHASH, 201, 5, 2, label="uniform")
    assert out[3][-1] > 100
    _check_batched(ctx, stations, 4096, 20, 4, fl.MINHASH, 201, 5, 2, distinct=True, label="uniform")


def test_batched_filter_uses_station_n(ctx):
    # Station 0 carries a repeating noise source (5 % of slots): its buckets
    # exceed 1 % of its own n and are excluded.  Station 1 is plain; station 2
    # is twice as long, so the same noise share is judged against its own n.
    stations = [
        synth.generate(synth.with_noise(synth.station(n=30_000, seed=41), 50, 190)),
        synth.generate(synth.station(n=20_000, seed=90)),
        synth.generate(synth.with_noise(synth.station(n=60_000, seed=91), 8, 190)),
    ]
    out = _check_batched(ctx, stations, 4096, 100, 4, fl.MINMAX, 42, 5, 4, 1, 100, label="filter")
    sts = out[4]
    assert sts[0].n_flagged > 1000 and sts[1].n_flagged == 0


def test_batched_minmax_groups_and_distinct(ctx):
    stations = [synth.generate(synth.station(n=n, seed=95 + n % 7)) for n in (40_000, 25_000, 15_000)]
    _check_batched(ctx, stations, 4096, 100, 4, fl.MINMAX, 202, 5, 4, 1, 100, label="minmax-v4")
    _check_batched(ctx, stations, 4096, 40, 4, fl.MINHASH, 33, 5, 3, distinct=True, label="minhash-v3-distinct")


@pytest.mark.parametrize("bits", [8, 16, 24, 32])
def test_batched_bin_bits(bits):
    """Bin bits of the tagged keys (station in the top four bits) change speed
    only: every choice gives each station's oracle output."""
    c = fl.FastLSH(0)
    c.configure(bin_bits=bits)
    stations = [synth.generate(synth.with_noise(synth.station(n=30_000, seed=41), 50, 190)),
                synth.generate(synth.station(n=50_000, seed=90)), _fixed(5, 4096, 200, 3)]
    _check_batched(c, stations, 4096, 100, 4, fl.MINMAX, 42, 5, 4, 1, 100, label=f"bin-bits-{bits}")
    bounded = c.search_bounded(fl.to_device_rows(stations[1]), 4096, 100, 4, fl.MINMAX, *fl.make_hash(42, 200), 5, 4,
                               1, 100, group_tables=10)
    full = c.search(fl.to_device_rows(stations[1]), 4096, 100, 4, fl.MINMAX, *fl.make_hash(42, 200), 5, 4, 1, 100)
    assert all(torch.equal(x, y) for x, y in zip(bounded[:3], full[:3])) and bounded[3] == full[3]
    c.close()


def test_batched_sixteen_stations(ctx):
    stations = [_fixed(300 + 137 * s, 256, 6, 700 + s) for s in range(16)]
    _check_batched(ctx, stations, 256, 12, 2, fl.MINMAX, 701, 2, 2, label="16-stations")
    _check_batched(ctx, stations, 256, 12, 2, fl.MINMAX, 701, 2, 2, 1, 50, distinct=True, label="16-stations")


def test_batched_one_station_equals_search(ctx):
    rows = synth.generate(synth.station(n=50_000, seed=102))
    a, b = fl.make_hash(202, 200)
    dev = fl.to_device_rows(rows)
    si, sj, sv, sst = ctx.search(dev, 4096, 100, 4, fl.MINMAX, a, b, 5, 4, 1, 100)
    bi, bj, bv, offs, bst = ctx.search_batched([dev], 4096, 100, 4, fl.MINMAX, a, b, 5, 4, 1, 100)
    assert torch.equal(si, bi) and torch.equal(sj, bj) and torch.equal(sv, bv)
    assert bst[0] == sst and offs.tolist() == [0, len(si)]


def test_batched_rejects_bad_input(ctx):
    a, b = fl.make_hash(1, 80)
    rows = fl.to_device_rows(_fixed(100, 4096, 20, 3))
    for stations in ([], [rows] * 17):
        with pytest.raises(fl.FastLshError) as e:
            ctx.search_batched(stations, 4096, 20, 4, fl.MINHASH, a, b, 5, 2)
        assert e.value.code == 1
    # 16-bit indices x 4 rows = 64 key bits: no room for the station tag
    wide = fl.to_device_rows(_fixed(100, 65536, 20, 4))
    with pytest.raises(fl.FastLshError) as e:
        ctx.search_batched([wide, wide], 65536, 20, 4, fl.MINHASH, a, b, 5, 2)
    assert e.value.code == 1
    ctx.search_batched([wide], 65536, 20, 4, fl.MINHASH, a, b, 5, 2)  # one station: untagged, allowed


def test_batched_capacity(ctx):
    stations = [synth.generate(synth.tiny_uniform(n=n, seed=61 + n)) for n in (20_000, 10_000)]
    a, b = fl.make_hash(62, 80)
    dev = [fl.to_device_rows(s) for s in stations]
    full = ctx.search_batched(dev, 4096, 20, 4, fl.MINHASH, a, b, 5, 1)
    assert full[3][-1] > 20
    with pytest.raises(fl.FastLshError) as e:
        ctx.search_batched(dev, 4096, 20, 4, fl.MINHASH, a, b, 5, 1, capacity=5)
    assert e.value.code == 3
    again = ctx.search_batched(dev, 4096, 20, 4, fl.MINHASH, a, b, 5, 1, capacity=None)
    for x, y in zip(full[:3], again[:3]):
        assert torch.equal(x, y)


# ---------------------------------------------------------------------------
# Captured graph: replays (with other eager work between them) and recaptures
# must reproduce the eager result every time.
# ---------------------------------------------------------------------------
def test_graph_replays_match_eager(ctx):
    rows = synth.generate(synth.station(n=60_000, seed=120))
    other = synth.generate(synth.tiny_uniform(n=15_000, seed=121))
    a, b = fl.make_hash(202, 200)
    dev = fl.to_device_rows(rows)
    say("[graph] eager reference")
    ref = ctx.search(dev, 4096, 100, 4, fl.MINMAX, a, b, 5, 4, 1, 100)
    for k in range(4):
        say(f"[graph] replay {k}")
        got = ctx.search(dev, 4096, 100, 4, fl.MINMAX, a, b, 5, 4, 1, 100, graph=True)
        for x, y in zip(ref[:3], got[:3]):
            assert torch.equal(x, y), k
        assert got[3] == ref[3]
        # eager work between replays: another search (other shapes) and torch ops
        a2, b2 = fl.make_hash(201, 80)
        ctx.search(fl.to_device_rows(other), 4096, 20, 4, fl.MINHASH, a2, b2, 5, 2)
        torch.cuda.synchronize()
        (dev.float() * 2).sum().item()
    # a second input buffer: recapture, still identical
    dev2 = fl.to_device_rows(rows)
    got = ctx.search(dev2, 4096, 100, 4, fl.MINMAX, a, b, 5, 4, 1, 100, graph=True)
    for x, y in zip(ref[:3], got[:3]):
        assert torch.equal(x, y)


def test_graph_replays_with_queue_overflow():
    """Graph replays whose pair launch overflows a one-entry candidate queue
    (the chunks run again after each replay), then the queue switched off
    (a new capture): every result equals the eager search's."""
    c = fl.FastLSH(0)
    try:
        rows = synth.generate(synth.with_noise(synth.station(n=30_000, seed=122), 50, 190))
        a, b = fl.make_hash(203, 200)
        dev = fl.to_device_rows(rows)
        say("[graph] eager reference, queue_slot=1")
        c.configure(queue_slot=1)
        ref = c.search(dev, 4096, 100, 4, fl.MINMAX, a, b, 5, 4)
        assert c.last_work()["pair_redos"] > 0
        for k in range(3):
            say(f"[graph] replay {k}, queue_slot=1")
            got = c.search(dev, 4096, 100, 4, fl.MINMAX, a, b, 5, 4, graph=True)
            assert all(torch.equal(x, y) for x, y in zip(ref[:3], got[:3])) and got[3] == ref[3], k
            assert c.last_work()["pair_redos"] > 0
            (dev.float() * 2).sum().item()
        say("[graph] queue off")
        c.configure(queue_slot=fl.QUEUE_OFF)
        got = c.search(dev, 4096, 100, 4, fl.MINMAX, a, b, 5, 4, graph=True)
        assert all(torch.equal(x, y) for x, y in zip(ref[:3], got[:3])) and got[3] == ref[3]
        assert c.last_work()["pair_redos"] == 0 and c.config_used()["queue_slot"] == fl.QUEUE_OFF
    finally:
        c.close()


def test_graph_batched_replays(ctx):
    stations = [synth.generate(synth.tiny_uniform(n=n, seed=1030 + n)) for n in (12_000, 30_000, 5_000)]
    for k in range(3):
        _check_batched(ctx, stations, 4096, 20, 4, fl.MINHASH, 201, 5, 2, graph=True, label=f"graph-{k}")


# ---------------------------------------------------------------------------
# Launch shapes change speed, never output bytes.
# ---------------------------------------------------------------------------
def test_launch_shapes_identical():
    c = fl.FastLSH(0)
    try:
        stations = [synth.generate(synth.station(n=n, seed=130 + n % 11)) for n in (70_000, 30_000)]
        a, b = fl.make_hash(202, 200)
        dev = [fl.to_device_rows(s) for s in stations]
        ref = c.search_batched(dev, 4096, 100, 4, fl.MINMAX, a, b, 5, 4, 1, 100)
        used = c.config_used()
        assert {k: used[k] for k in ("radix_tile", "bucket_chunk", "autotune")} == \
            {"radix_tile": 16384, "bucket_chunk": 512, "autotune": False}
        assert used["bin_bits"] == 24  # 70,000 fingerprints: 15 bits plus the four station bits, two passes
        for tile in (16384, 8192, 4096):
            for chunk in (256, 768, 1024, 1536):
                say(f"[shapes] radix_tile={tile} bucket_chunk={chunk}")
                c.configure(radix_tile=tile, bucket_chunk=chunk)
                got = c.search_batched(dev, 4096, 100, 4, fl.MINMAX, a, b, 5, 4, 1, 100)
                assert c.config_used()["radix_tile"] == tile and c.config_used()["bucket_chunk"] == chunk
                for x, y in zip(ref[:3], got[:3]):
                    assert torch.equal(x, y)
                assert (ref[3] == got[3]).all() and ref[4] == got[4]
        c.configure(autotune=True)
        for k in range(2):  # the first call tunes, the second reuses the choice
            say(f"[shapes] autotune call {k}")
            got = c.search_batched(dev, 4096, 100, 4, fl.MINMAX, a, b, 5, 4, 1, 100, graph=(k == 1))
            used = c.config_used()
            assert used["radix_tile"] in (16384, 8192, 4096) and used["bucket_chunk"] in (256, 512, 768, 1024)
            for x, y in zip(ref[:3], got[:3]):
                assert torch.equal(x, y)
            assert ref[4] == got[4]
        with pytest.raises(fl.FastLshError):
            c.configure(radix_tile=1000)
        with pytest.raises(fl.FastLshError):
            c.configure(bucket_chunk=2048)
    finally:
        c.close()


# ---------------------------------------------------------------------------
# Bounded-memory search: identical output and counters to the full search
# (and to the oracle) for every table-group size.
# ---------------------------------------------------------------------------
BOUNDED = [
    ("station-g10", lambda: synth.generate(synth.station(n=120_000, seed=150)), 4096, 100, 4, fl.MINMAX, 5, 4, 1, 100, 10),
    ("station-g7", lambda: synth.generate(synth.station(n=60_000, seed=151)), 4096, 100, 4, fl.MINMAX, 5, 4, 1, 100, 7),
    ("station-g1", lambda: synth.generate(synth.station(n=20_000, seed=152)), 4096, 30, 4, fl.MINMAX, 5, 3, 1, 100, 1),
    ("noise-g13", lambda: synth.generate(synth.with_noise(synth.station(n=30_000, seed=41), 50, 190)), 4096, 100, 4,
     fl.MINMAX, 5, 4, 1, 100, 13),
    ("noise-nofilter-g34", lambda: synth.generate(synth.with_noise(synth.station(n=30_000, seed=42), 50, 190)), 4096,
     100, 4, fl.MINMAX, 5, 4, 0, 0, 34),
    ("uniform-minhash-g6", lambda: synth.generate(synth.tiny_uniform()), 4096, 20, 4, fl.MINHASH, 5, 2, 0, 0, 6),
    ("ragged-g5", lambda: _ragged_rows(3000, 512, 1, 40, 56), 512, 12, 2, fl.MINMAX, 3, 2, 0, 0, 5),
    ("identical-g2", lambda: np.repeat(_fixed(1, 4096, 200, 43), 3000, axis=0), 4096, 5, 4, fl.MINMAX, 100, 2, 0, 0, 2),
]


def _ragged_rows(n, dim, lo, hi, seed):
    rng = np.random.default_rng(seed)
    lens = rng.integers(lo, hi + 1, n)
    rows = [np.sort(rng.choice(dim, L, replace=False)).astype(np.uint16) for L in lens]
    return np.concatenate(rows), np.concatenate([[0], np.cumsum(lens)]).astype(np.uint64)


def _dev(rows):
    if isinstance(rows, tuple):
        ind, off = rows
        return (torch.from_numpy(ind.view(np.int16)).cuda(), torch.from_numpy(off.view(np.int64)).cuda())
    return fl.to_device_rows(rows)


@pytest.mark.parametrize("name,make,dim,t,r,scheme,L,v,num,den,gt", BOUNDED, ids=[b[0] for b in BOUNDED])
def test_bounded_matches_full_and_oracle(ctx, name, make, dim, t, r, scheme, L, v, num, den, gt):
    rows = make()
    a, b = fl.make_hash(205, fl.n_funcs(t, r, scheme))
    dev = _dev(rows)
    ngroups = -(-t // gt)
    for distinct in (False, True):
        full = ctx.search(dev, dim, t, r, scheme, a, b, L, v, num, den, want_distinct=distinct)
        # pass 2 on pass 1's kept groupings (all of them: HBM holds these
        # sizes), on none (every group sorted again), and on the first only
        for keep in (fl.KEEP_AUTO, 0, 1):
            say(f"[bounded] {name} group_tables={gt} distinct={distinct} keep_groups={keep:#x}")
            ctx.configure(keep_groups=keep)
            bnd = ctx.search_bounded(dev, dim, t, r, scheme, a, b, L, v, num, den, group_tables=gt,
                                     want_distinct=distinct)
            assert ctx.config_used()["keep_groups"] == (ngroups if keep == fl.KEEP_AUTO else min(keep, ngroups))
            for x, y in zip(full[:3], bnd[:3]):
                assert torch.equal(x, y)
            assert full[3] == bnd[3]
    ctx.configure()
    ei, ej, ev, est = oracle.search(rows, dim, t, r, scheme, a, b, L, v, num, den)
    assert np.array_equal(_np(bnd[0], np.uint32), ei) and np.array_equal(_np(bnd[1], np.uint32), ej)
    assert np.array_equal(bnd[2].cpu().numpy(), ev)
    want = dict(est.__dict__)
    got = dict(bnd[3].__dict__)
    want.pop("n_distinct")
    got.pop("n_distinct")
    assert got == want


def test_bounded_rejects(ctx):
    a, b = fl.make_hash(1, 80)
    rows = fl.to_device_rows(_fixed(100, 65536, 20, 4))
    with pytest.raises(fl.FastLshError) as e:  # 64-bit band keys
        ctx.search_bounded(rows, 65536, 20, 4, fl.MINHASH, a, b, 5, 2)
    assert e.value.code == 1
    rows = fl.to_device_rows(_fixed(100, 4096, 20, 5))
    with pytest.raises(fl.FastLshError) as e:
        ctx.search_bounded(rows, 4096, 20, 4, fl.MINHASH, a, b, 5, 2, group_tables=0)
    assert e.value.code == 1
    empty = torch.empty((0, 200), dtype=torch.int16, device="cuda")
    gi, gj, gv, st = ctx.search_bounded(empty, 4096, 20, 4, fl.MINHASH, a, b, 5, 2)
    assert len(gi) == 0 and st.n_out == 0


def test_bounded_keeps_what_the_budget_holds():
    # A context whose HBM budget holds the bounded search's workspace plus
    # about two and a half groups' kept groupings keeps one or two of the ten
    # and sorts the others again; the result is the full search's either way.
    rows = synth.generate(synth.station(n=3_000_000, seed=48))
    a, b = fl.make_hash(205, 200)
    dev = fl.to_device_rows(rows)
    args = (dev, 4096, 100, 4, fl.MINMAX, a, b, 5, 4, 1, 100)
    c0 = fl.FastLSH(0)
    full = c0.search(*args)
    c0.close()
    sizes = {}
    for keep in (0, fl.KEEP_AUTO):
        c = fl.FastLSH(0)
        c.configure(keep_groups=keep, queue_slot=fl.QUEUE_OFF)  # (a budget context has no automatic queue)
        out = c.search_bounded(*args, group_tables=10)
        sizes[keep] = (c.workspace_bytes(), c.config_used()["keep_groups"])
        c.close()
        for x, y in zip(full[:3], out[:3]):
            assert torch.equal(x, y)
        assert full[3] == out[3]
    assert sizes[0][1] == 0 and sizes[fl.KEEP_AUTO][1] == 10
    per_group = (sizes[fl.KEEP_AUTO][0] - sizes[0][0]) / 10
    budget = int(sizes[0][0] + 2.5 * per_group)
    say(f"[bounded] workspace {sizes[0][0]} without kept groupings, {per_group:.0f} per kept group; budget {budget}")
    c = fl.FastLSH(0, hbm_budget=budget)
    out = c.search_bounded(*args, group_tables=10)
    kept = c.config_used()["keep_groups"]
    assert 1 <= kept <= 2 and c.workspace_bytes() <= budget
    c.close()
    say(f"[bounded] budget keeps {kept} groupings")
    for x, y in zip(full[:3], out[:3]):
        assert torch.equal(x, y)
    assert full[3] == out[3]
