"""GPU parity: the HIP path through the C-ABI against the CPU oracle.

Every comparison is exact (integers only): band keys and hash values bit for
bit, pair lists (i, j, votes) element by element, and all counters.
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


def _u64(t):
    return t.cpu().numpy().view(np.uint64)


def _rows_dev(rows):
    if isinstance(rows, tuple):
        ind, off = rows
        return (torch.from_numpy(ind.view(np.int16)).cuda(), torch.from_numpy(off.view(np.int64)).cuda())
    return fl.to_device_rows(rows)


# ---------------------------------------------------------------------------
# Hash parameters and signatures
# ---------------------------------------------------------------------------
def test_make_hash_matches_oracle():
    for seed in (0, 201, 202, 2**63 + 5):
        a, b = fl.make_hash(seed, 1000)
        oa, ob = oracle.make_hash(seed, 1000)
        assert (a == oa).all() and (b == ob).all()


def _ragged(n, dim, lo, hi, seed):
    rng = np.random.default_rng(seed)
    lens = rng.integers(lo, hi + 1, n)
    rows = [np.sort(rng.choice(dim, L, replace=False)).astype(np.uint16) for L in lens]
    return np.concatenate(rows), np.concatenate([[0], np.cumsum(lens)]).astype(np.uint64)


def _fixed(n, dim, nnz, seed):
    rng = np.random.default_rng(seed)
    return np.stack([np.sort(rng.choice(dim, nnz, replace=False)) for _ in range(n)]).astype(np.uint16)


SIG_CASES = [
    # name, rows factory, dim, t, r, scheme
    ("station-minmax-nnz200", lambda: synth.generate(synth.station(n=3000, seed=11)), 4096, 100, 4, fl.MINMAX),
    ("uniform-minhash-nnz200", lambda: synth.generate(synth.tiny_uniform(n=3001, seed=12)), 4096, 20, 4, fl.MINHASH),
    ("nnz100-dword-path", lambda: _fixed(777, 4096, 100, 13), 4096, 30, 4, fl.MINMAX),
    ("nnz16", lambda: _fixed(300, 1000, 16, 14), 1000, 8, 2, fl.MINHASH),
    ("nnz37-odd-long-path", lambda: _fixed(500, 4096, 37, 15), 4096, 12, 4, fl.MINHASH),
    ("nnz300-long-path", lambda: _fixed(200, 4096, 300, 16), 4096, 10, 4, fl.MINMAX),
    ("ragged", lambda: _ragged(400, 2048, 1, 90, 17), 2048, 16, 4, fl.MINMAX),
    ("dim16-r3", lambda: _fixed(300, 16, 6, 18), 16, 9, 3, fl.MINHASH),
    ("dim65536-r4-full64", lambda: _fixed(300, 65536, 64, 19), 65536, 7, 4, fl.MINMAX),
    ("dim8192-r8-chained", lambda: _fixed(300, 8192, 128, 20), 8192, 6, 8, fl.MINMAX),
    # eight functions per pass over a row: one function per table, and three
    # (passes that end inside a table)
    ("minhash-r1", lambda: _fixed(500, 4096, 200, 25), 4096, 13, 1, fl.MINHASH),
    ("minmax-r6-chained", lambda: _fixed(400, 4096, 200, 26), 4096, 7, 6, fl.MINMAX),
]


@pytest.mark.parametrize("name,make,dim,t,r,scheme", SIG_CASES, ids=[c[0] for c in SIG_CASES])
def test_signatures_bit_exact(ctx, name, make, dim, t, r, scheme):
    rows = make()
    say(f"[sig] {name}")
    nf = fl.n_funcs(t, r, scheme)
    a, b = fl.make_hash(900 + t * r, nf)
    keys, vals = ctx.signatures(_rows_dev(rows), dim, t, r, scheme, a, b, with_values=True)
    torch.cuda.synchronize()
    okeys, ovals = oracle.signatures(rows, dim, t, r, scheme, a, b, with_values=True)
    assert np.array_equal(_u64(keys), okeys)
    assert np.array_equal(vals.cpu().numpy().view(np.uint32), ovals)


FOLD_CASES = [(200, fl.MINMAX), (200, fl.MINHASH), (100, fl.MINMAX), (300, fl.MINMAX), (37, fl.MINHASH)]


@pytest.mark.parametrize("nnz,scheme", FOLD_CASES, ids=[f"nnz{c[0]}-{'minmax' if c[1] == fl.MINMAX else 'minhash'}" for c in FOLD_CASES])
def test_signatures_fold_edge_values(ctx, nnz, scheme):
    """Hash parameters chosen so that every function reaches a residue k in
    0..7 at the largest index of one fingerprint, from a y = a x + b of many
    multiples of p.  Folding y to (y mod 2^31) + (y >> 31) then gives p itself
    (k = 0) or a value of at least 2^31 (k > 0): the two forms whose
    canonical residue needs the correction step."""
    dim, t, r = 4096, 12, 4
    P = 2**31 - 1
    rows = _fixed(300, dim, nnz, 23 + nnz)
    nf = fl.n_funcs(t, r, scheme)
    a, _ = fl.make_hash(77 + nnz, nf)
    b = np.empty(nf, np.uint32)
    hit = 0
    for f in range(nf):
        x0 = int(rows[f % len(rows)].max())
        k = f % 8
        b[f] = (k - int(a[f]) * x0) % P
        y = int(a[f]) * x0 + int(b[f])
        s = (y & P) + (y >> 31)
        hit += s >= P
    assert hit == nf  # every function has its out-of-range fold
    say(f"[sig-fold] nnz={nnz} scheme={scheme}")
    keys, vals = ctx.signatures(fl.to_device_rows(rows), dim, t, r, scheme, a, b, with_values=True)
    torch.cuda.synchronize()
    okeys, ovals = oracle.signatures(rows, dim, t, r, scheme, a, b, with_values=True)
    assert np.array_equal(_u64(keys), okeys)
    assert np.array_equal(vals.cpu().numpy().view(np.uint32), ovals)


def test_signatures_table_range(ctx):
    rows = synth.generate(synth.station(n=1000, seed=21))
    a, b = fl.make_hash(5, 100)
    okeys = oracle.signatures(rows, 4096, 50, 4, oracle.MINMAX, a, b)
    keys = ctx.signatures(_rows_dev(rows), 4096, 50, 4, fl.MINMAX, a, b, table_begin=17, table_count=9)
    assert np.array_equal(_u64(keys), okeys[17:26])


def test_signatures_reject_bad_input(ctx):
    a, b = fl.make_hash(1, 40)
    bad = _fixed(64, 4096, 200, 22)
    bad[10, 5] = 4096  # index >= dim
    with pytest.raises(fl.FastLshError) as e:
        ctx.signatures(_rows_dev(bad), 4096, 20, 4, fl.MINMAX, a, b)
    assert e.value.code == 1
    ind, off = _ragged(50, 512, 1, 10, 23)
    off[7] = off[8]  # empty row 7
    off = off.copy()
    with pytest.raises(fl.FastLshError):
        ctx.signatures(_rows_dev((ind, off)), 512, 20, 4, fl.MINMAX, a, b)
    with pytest.raises(fl.FastLshError):
        ctx.signatures(_rows_dev(_fixed(10, 64, 4, 24)), 64, 20, 3, fl.MINMAX, a, b)  # odd r, Min-Max
    bad_a = a.copy()
    bad_a[3] = 0
    with pytest.raises(fl.FastLshError):
        ctx.signatures(_rows_dev(_fixed(10, 64, 4, 24)), 64, 20, 4, fl.MINMAX, bad_a, b)


# ---------------------------------------------------------------------------
# Search
# ---------------------------------------------------------------------------
def _compare(ctx, rows, dim, t, r, scheme, seed, L, v, num=0, den=0, distinct=False, label=""):
    say(f"[search] {label} n={len(rows) if not isinstance(rows, tuple) else len(rows[1]) - 1} t={t} r={r} "
        f"scheme={scheme} L={L} v={v} occ={num}/{den} distinct={distinct}")
    nf = fl.n_funcs(t, r, scheme)
    a, b = fl.make_hash(seed, nf)
    gi, gj, gv, gst = ctx.search(_rows_dev(rows), dim, t, r, scheme, a, b, L, v, num, den, want_distinct=distinct)
    torch.cuda.synchronize()
    keys = oracle.signatures(rows, dim, t, r, scheme, a, b)
    ei, ej, ev, est = oracle.search_keys(keys, L, v, num, den)
    gi = gi.cpu().numpy().view(np.uint32)
    gj = gj.cpu().numpy().view(np.uint32)
    gv = gv.cpu().numpy()
    assert len(gi) == len(ei), (len(gi), len(ei))
    assert np.array_equal(gi, ei)
    assert np.array_equal(gj, ej)
    assert np.array_equal(gv, ev)
    want = dict(est.__dict__)
    got = dict(gst.__dict__)
    if not distinct:
        assert got.pop("n_distinct") == 2**64 - 1
        want.pop("n_distinct")
    assert got == want
    return gst


@pytest.mark.parametrize("n,num,den,keep,drop", [(1000, 1, 100, 10, 11), (1050, 1, 100, 10, 11),
                                                 (1000, 3, 1000, 3, 4)])
def test_search_occurrence_bound(ctx, n, num, den, keep, drop):
    """Section 6.5: a bucket is excluded when its members exceed num / den of
    the fingerprints.  `keep` identical fingerprints (a bucket of that size in
    every table, exactly floor(n num / den)) stay; `drop` identical ones go."""
    rows = _fixed(n, 4096, 200, 27 + n + num)
    rows[100:100 + keep] = rows[100]
    rows[500:500 + drop] = rows[500]
    st = _compare(ctx, rows, 4096, 20, 4, fl.MINMAX, 28, 1, 4, num, den, label=f"occ-bound-{n}-{num}/{den}")
    assert st.n_flagged == drop
    assert st.n_out >= keep * (keep - 1) // 2


def test_search_tiny_uniform_full(ctx):
    rows = synth.generate(synth.tiny_uniform())
    st = _compare(ctx, rows, 4096, 20, 4, fl.MINHASH, 201, 5, 2, label="tiny-uniform-20k")
    assert st.n_out > 50
    _compare(ctx, rows, 4096, 20, 4, fl.MINHASH, 201, 5, 2, distinct=True, label="tiny-uniform-20k")


@pytest.mark.parametrize("n", [50_000, 200_000, 400_000])
def test_search_station(ctx, n):
    # 400,000 fingerprints bin on 24 key bits (three radix passes), as the
    # 90-day station does; 200,000 on 16 (two passes)
    rows = synth.generate(synth.station(n=n, seed=102))
    st = _compare(ctx, rows, 4096, 100, 4, fl.MINMAX, 202, 5, 4, 1, 100, label="station")
    assert st.n_out > 0
    if n != 200_000:
        _compare(ctx, rows, 4096, 100, 4, fl.MINMAX, 202, 5, 4, 1, 100, distinct=True, label="station")


@pytest.mark.parametrize("bits,n,t,seed", [(8, 120_000, 100, 61), (24, 120_000, 100, 61), (32, 120_000, 100, 61),
                                          (8, 50_000, 2, 90), (8, 50_000, 100, 90)])
def test_search_bin_bits(bits, n, t, seed):
    """The grouping passes' bin bits change speed only: coarser or finer bins
    give the oracle's output and counters (the automatic choice here is 16).
    With 8 bits and 50,000 fingerprints some table's last bin holds 193-256
    members and runs to the table's end, the case where the bucket kernel
    once took the bin's end past the table (into the next one)."""
    c = fl.FastLSH(0)
    c.configure(bin_bits=bits)
    spec = synth.station(n=n, seed=seed)
    rows = synth.generate(synth.with_noise(spec, 20, 190) if seed == 61 else spec)
    _compare(c, rows, 4096, t, 4, fl.MINMAX, 62 if seed == 61 else 42, 5, 4 if t > 2 else 1, 1, 100,
             label=f"bin-bits-{bits}")
    assert c.config_used()["bin_bits"] == bits
    c.close()


def test_search_station_minhash_v3(ctx):
    rows = synth.generate(synth.station(n=60_000, seed=31))
    _compare(ctx, rows, 4096, 40, 4, fl.MINHASH, 33, 5, 3, label="station-minhash")


@pytest.mark.parametrize("num,den", [(1, 100), (0, 0)])
def test_search_repeating_noise(ctx, num, den):
    # 5 % of slots are 95 %-copies of one noise template: huge buckets that the
    # occurrence filter removes, or (filter off) the large-bucket tile path.
    rows = synth.generate(synth.with_noise(synth.station(n=30_000, seed=41), 50, 190))
    st = _compare(ctx, rows, 4096, 100, 4, fl.MINMAX, 42, 5, 4, num, den, label="noise")
    assert st.max_bucket > 300
    if den:
        assert st.n_flagged > 1000


@pytest.mark.parametrize("qslot,v", [(0, 4), (1, 4), (3, 4), (fl.QUEUE_OFF, 4), (1, 2), (0, 2)])
def test_search_candidate_queue(qslot, v):
    """The pair kernels queue the pairs that pass the sub-key group test and
    check them in a later launch; a workgroup whose queue slot fills up runs
    again with the checks in place.  Any queue size gives the oracle's
    output and counters: one entry per slot forces the second runs (tiled
    and small-bucket launches), QUEUE_OFF checks everything in place.  v=4
    splits 100 tables into 3 groups (17-dword rows, the checks take the
    rows' field masks), v=2 keeps one group (50-dword rows)."""
    c = fl.FastLSH(0)
    c.configure(queue_slot=qslot)
    rows = synth.generate(synth.with_noise(synth.station(n=30_000, seed=47), 50, 190))
    st = _compare(c, rows, 4096, 100, 4, fl.MINMAX, 48, 5, v, label=f"queue-{qslot}")
    assert st.max_bucket > 300
    used = c.config_used()["queue_slot"]
    assert used == (qslot if qslot else 30_000 // 64 if 30_000 // 64 > 64 else 64)
    redos = c.last_work()["pair_redos"]
    assert redos == 0 if qslot == fl.QUEUE_OFF else (redos > 0 if qslot == 1 else True)
    c.close()


def test_search_queue_under_budget():
    """A context with an HBM budget searches without the automatic candidate
    queue (checks in place, same result, the same workspace as with the
    queue off); a queue size asked for that does not fit is E_NOMEM."""
    rows = synth.generate(synth.with_noise(synth.station(n=30_000, seed=51), 50, 190))
    a, b = fl.make_hash(52, fl.n_funcs(100, 4, fl.MINMAX))
    free = fl.FastLSH(0)
    free.configure(queue_slot=fl.QUEUE_OFF)
    ref = free.search(fl.to_device_rows(rows), 4096, 100, 4, fl.MINMAX, a, b, 5, 4)
    need = free.workspace_bytes()
    free.close()
    c = fl.FastLSH(0, hbm_budget=need + (1 << 20))
    try:
        say(f"[search] budget {need + (1 << 20)} bytes, automatic queue")
        got = c.search(fl.to_device_rows(rows), 4096, 100, 4, fl.MINMAX, a, b, 5, 4)
        assert all(torch.equal(x, y) for x, y in zip(ref[:3], got[:3])) and got[3] == ref[3]
        assert c.config_used()["queue_slot"] == fl.QUEUE_OFF and c.workspace_bytes() == need
        c.configure(queue_slot=16384)  # 256 MiB of queue
        with pytest.raises(fl.FastLshError) as e:
            c.search(fl.to_device_rows(rows), 4096, 100, 4, fl.MINMAX, a, b, 5, 4)
        assert e.value.code == fl.E_NOMEM
    finally:
        c.close()


def test_bounded_candidate_queue_overflow():
    """The bounded search with one queue entry per slot (second runs in
    every pair launch of both passes' groups) against the oracle."""
    c = fl.FastLSH(0)
    c.configure(queue_slot=1)
    rows = synth.generate(synth.with_noise(synth.station(n=30_000, seed=49), 50, 190))
    a, b = fl.make_hash(50, fl.n_funcs(100, 4, fl.MINMAX))
    say("[search] bounded queue_slot=1 n=30000 t=100 v=4 groups of 10")
    gi, gj, gv, gst = c.search_bounded(fl.to_device_rows(rows), 4096, 100, 4, fl.MINMAX, a, b, 5, 4, 1, 100,
                                       group_tables=10)
    assert c.last_work()["pair_redos"] > 0
    keys = oracle.signatures(rows, 4096, 100, 4, fl.MINMAX, a, b)
    ei, ej, ev, est = oracle.search_keys(keys, 5, 4, 1, 100)
    assert np.array_equal(gi.cpu().numpy().view(np.uint32), ei)
    assert np.array_equal(gj.cpu().numpy().view(np.uint32), ej)
    assert np.array_equal(gv.cpu().numpy(), ev)
    got, want = dict(gst.__dict__), dict(est.__dict__)
    assert got.pop("n_distinct") == 2**64 - 1
    want.pop("n_distinct")
    assert got == want
    with pytest.raises(fl.FastLshError):
        c.configure(queue_slot=(1 << 20) + 1)
    c.close()


def test_search_huge_bins(ctx):
    # Every fingerprint identical: one bucket of n in every table (oversized
    # bins, the single-workgroup sort path and tiled pairs).
    rows = np.repeat(_fixed(1, 4096, 200, 43), 5000, axis=0)
    st = _compare(ctx, rows, 4096, 3, 4, fl.MINMAX, 44, 100, 2, label="identical")
    assert st.max_bucket == 5000 and st.n_out == (5000 - 100) * (5000 - 99) // 2


def test_search_mixed_huge_bins(ctx):
    # Half the rows identical (one giant bucket per table), the rest random:
    # oversized bins that also hold other keys.
    rows = _fixed(9000, 256, 8, 45)
    rows[::2] = rows[0]
    _compare(ctx, rows, 256, 4, 2, fl.MINHASH, 46, 1, 2, label="mixed-identical")


def _near_copies(n_base, copies, dim, nnz, lo, hi, seed):
    """Each base row and `copies` variants with lo..hi of its indices
    replaced (Jaccard about 0.3-0.5: pairs sharing a handful of tables),
    in random order."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n_base):
        base = rng.choice(dim, nnz, replace=False)
        out.append(np.sort(base))
        for _ in range(copies):
            k = int(rng.integers(lo, hi + 1))
            keep = rng.choice(base, nnz - k, replace=False)
            pool = np.setdiff1d(np.arange(dim), base)
            out.append(np.sort(np.concatenate([keep, rng.choice(pool, k, replace=False)])))
    rows = np.stack(out).astype(np.uint16)
    return rows[rng.permutation(len(rows))]


@pytest.mark.parametrize("t", [99, 100, 101])
def test_search_group_rows_near_threshold(ctx, t):
    # v = 4 puts t = 99..101 tables into 3 groups of 33-34 (the last one
    # shorter).  Copies of moderate similarity give many pairs just at the
    # vote threshold, where the owner rule turns on one or two shared tables
    # of a group, often in its last fields.
    rows = _near_copies(1500, 3, 4096, 200, 60, 110, 300 + t)
    st = _compare(ctx, rows, 4096, t, 4, fl.MINMAX, 61 + t, 2, 4, label=f"near-copies-t{t}")
    assert st.n_out > 500
    _compare(ctx, rows, 4096, t, 4, fl.MINMAX, 61 + t, 2, 4, distinct=True, label=f"near-copies-t{t}")


@pytest.mark.parametrize("v", [2, 4])
def test_search_long_and_mixed_bins(ctx, v):
    # 1,015 rows leave 8 bin bits, so the bins of groups of identical rows
    # (40-140 copies each) also hold other groups and single rows: bins that
    # mix keys below 64 members (ranked in the window), between 64 and 128
    # (ranked from HBM), above 128 (handed to the big-bin kernel), and
    # one-key bins longer than the 64-position window.
    sizes = [40, 45, 50, 60, 70, 80, 100, 130, 140]
    base = _fixed(len(sizes), 4096, 200, 90)
    rows = np.concatenate([np.repeat(base[g:g + 1], z, axis=0) for g, z in enumerate(sizes)] +
                          [_fixed(300, 4096, 200, 91)])
    rows = rows[np.random.default_rng(92).permutation(len(rows))]
    st = _compare(ctx, rows, 4096, 255, 4, fl.MINMAX, 93, 3, v, label=f"long-mixed-bins-v{v}")
    assert st.max_bucket >= 140 and st.n_out > 30_000
    _compare(ctx, rows, 4096, 255, 4, fl.MINMAX, 93, 3, v, distinct=True, label=f"long-mixed-bins-v{v}")


EDGE = [
    ("n1", lambda: _fixed(1, 4096, 200, 50), 4096, 10, 4, fl.MINMAX, 5, 2),
    ("n2-identical", lambda: np.repeat(_fixed(1, 4096, 200, 51), 2, axis=0), 4096, 10, 4, fl.MINMAX, 1, 10),
    ("t1-v1", lambda: _fixed(3000, 64, 4, 52), 64, 1, 2, fl.MINHASH, 0, 1),
    ("v1-lag0", lambda: _fixed(2000, 128, 6, 53), 128, 8, 2, fl.MINMAX, 0, 1),
    ("v-above-t", lambda: _fixed(2000, 128, 6, 54), 128, 3, 2, fl.MINMAX, 0, 4),
    ("lag-huge", lambda: _fixed(2000, 128, 6, 55), 128, 8, 2, fl.MINMAX, 1500, 1),
    ("ragged", lambda: _ragged(3000, 512, 1, 40, 56), 512, 12, 2, fl.MINMAX, 3, 2),
    ("odd-nnz", lambda: _fixed(3000, 256, 7, 57), 256, 12, 2, fl.MINHASH, 3, 3),
    ("t255", lambda: _fixed(1500, 128, 5, 58), 128, 255, 1, fl.MINHASH, 2, 30),
]


@pytest.mark.parametrize("name,make,dim,t,r,scheme,L,v", EDGE, ids=[e[0] for e in EDGE])
def test_search_edge_cases(ctx, name, make, dim, t, r, scheme, L, v):
    rows = make()
    _compare(ctx, rows, dim, t, r, scheme, 60, L, v, label=name)
    _compare(ctx, rows, dim, t, r, scheme, 60, L, v, distinct=True, label=name)


def test_search_empty(ctx):
    a, b = fl.make_hash(1, 40)
    empty = torch.empty((0, 200), dtype=torch.int16, device="cuda")
    gi, gj, gv, st = ctx.search(empty, 4096, 20, 2, fl.MINHASH, a, b, 5, 2)
    assert len(gi) == 0 and st.n_out == 0 and st.e_raw == 0


def test_search_capacity_and_copy(ctx):
    rows = synth.generate(synth.tiny_uniform(n=20_000, seed=61))
    a, b = fl.make_hash(62, 80)
    gi, gj, gv, st = ctx.search(fl.to_device_rows(rows), 4096, 20, 4, fl.MINHASH, a, b, 5, 1)
    assert st.n_out > 10
    with pytest.raises(fl.FastLshError) as e:
        ctx.search(fl.to_device_rows(rows), 4096, 20, 4, fl.MINHASH, a, b, 5, 1, capacity=5)
    assert e.value.code == 3
    # the result stays in the context: copy it into a large enough buffer
    cap = st.n_out
    oi = torch.empty(cap, dtype=torch.int32, device="cuda")
    oj = torch.empty(cap, dtype=torch.int32, device="cuda")
    ov = torch.empty(cap, dtype=torch.uint8, device="cuda")
    rc = fl.library().fast_lsh_copy_result(ctx._ctx, oi.data_ptr(), oj.data_ptr(), ov.data_ptr(), cap)
    assert rc == 0
    assert torch.equal(oi, gi) and torch.equal(oj, gj) and torch.equal(ov, gv)


def test_search_deterministic(ctx):
    rows = synth.generate(synth.station(n=100_000, seed=71))
    a, b = fl.make_hash(72, 200)
    outs = [ctx.search(fl.to_device_rows(rows), 4096, 100, 4, fl.MINMAX, a, b, 5, 4, 1, 100) for _ in range(2)]
    for x, y in zip(outs[0][:3], outs[1][:3]):
        assert torch.equal(x, y)
    assert outs[0][3] == outs[1][3]


def test_search_rejects_bad_input(ctx):
    a, b = fl.make_hash(1, 40)
    bad = _fixed(100, 4096, 200, 81)
    bad[3, 0] = 5000
    with pytest.raises(fl.FastLshError) as e:
        ctx.search(fl.to_device_rows(bad), 4096, 20, 2, fl.MINHASH, a, b, 5, 2)
    assert e.value.code == 1
    with pytest.raises(fl.FastLshError):
        ctx.search(fl.to_device_rows(_fixed(10, 4096, 200, 82)), 4096, 20, 2, fl.MINHASH, a, b, 5, 0)
