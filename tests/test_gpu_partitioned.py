"""GPU parity of the partitioned search with the dynamic occurrence filter
(sections 6.4, 6.5) through the C-ABI, against the oracle element by element
and counter by counter; without the filter, against the plain search."""
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


def _u32(t):
    return t.cpu().numpy().view(np.uint32)


def _compare(ctx, rows, t, r, scheme, seed, L, v, num, den, parts, distinct=False, label=""):
    say(f"[partitioned] {label}: n={len(rows)} t={t} L={L} v={v} occ={num}/{den} parts={parts} distinct={distinct}")
    a, b = fl.make_hash(seed, fl.n_funcs(t, r, scheme))
    gi, gj, gv, gst = ctx.search_partitioned(fl.to_device_rows(rows), 4096, t, r, scheme, a, b, L, v, num, den,
                                             n_partitions=parts, want_distinct=distinct)
    keys = oracle.signatures(rows, 4096, t, r, scheme, a, b)
    wi, wj, wv, wst = oracle.search_partitioned_keys(keys, L, v, num, den, min(parts, max(len(rows), 1)))
    assert np.array_equal(_u32(gi), wi) and np.array_equal(_u32(gj), wj) and np.array_equal(gv.cpu().numpy(), wv)
    got, want = dict(gst.__dict__), dict(wst.__dict__)
    if not distinct:
        assert got.pop("n_distinct") == 2**64 - 1
        want.pop("n_distinct")
    assert got == want, (got, want)
    return gst


@pytest.mark.parametrize("parts", [1, 3, 7])
def test_partitioned_without_filter_is_the_plain_search(ctx, parts):
    rows = synth.generate(synth.station(n=40_000, seed=81))
    a, b = fl.make_hash(82, 200)
    plain = ctx.search(fl.to_device_rows(rows), 4096, 100, 4, fl.MINMAX, a, b, 5, 4)
    part = ctx.search_partitioned(fl.to_device_rows(rows), 4096, 100, 4, fl.MINMAX, a, b, 5, 4, n_partitions=parts)
    assert all(torch.equal(x, y) for x, y in zip(plain[:3], part[:3])) and plain[3] == part[3]
    _compare(ctx, rows, 100, 4, fl.MINMAX, 82, 5, 4, 0, 0, parts, label="no filter")


@pytest.mark.parametrize("parts,num,den,t,v,distinct", [(1, 1, 100, 100, 4, False), (2, 1, 100, 100, 4, True),
                                                        (3, 1, 50, 16, 2, False), (5, 3, 100, 40, 3, False),
                                                        (4, 1, 100, 100, 1, True)])
def test_partitioned_filter_matches_oracle(ctx, parts, num, den, t, v, distinct):
    # repeating noise in part of the station: its fingerprints and their
    # neighbours go, partition by partition
    rows = synth.generate(synth.with_noise(synth.station(n=30_000, seed=83 + parts), 40, 190))
    st = _compare(ctx, rows, t, 4, fl.MINMAX, 84, 5, v, num, den, parts, distinct, label="noise")
    assert st.n_flagged > 100


def test_partitioned_station_months(ctx):
    # three "months" of a station with a burst of repeating noise in the second
    rows = synth.generate(synth.station(n=150_000, seed=85))
    noise = synth.generate(synth.with_noise(synth.station(n=20_000, seed=86), 300, 190))
    rows[60_000:80_000] = noise
    st = _compare(ctx, rows, 100, 4, fl.MINMAX, 87, 5, 4, 1, 100, 3, label="months")
    assert st.n_flagged > 1000


def test_partitioned_bursts_in_separate_partitions(ctx):
    # seven partitions of 10,000 with bursts of repeating noise in the second
    # and the fifth: the counting pass is taken again after each excluding
    # partition, and the pairs are reported in three runs (partition 0,
    # partitions 1-3, partitions 4-6), each with the exclusions of its time
    rows = synth.generate(synth.station(n=70_000, seed=90))
    for lo, seed in ((10_000, 91), (40_000, 92)):
        rows[lo:lo + 8_000] = synth.generate(synth.with_noise(synth.station(n=8_000, seed=seed), 200, 190))
    st = _compare(ctx, rows, 100, 4, fl.MINMAX, 93, 5, 4, 1, 100, 7, label="bursts in partitions 1 and 4")
    assert st.n_flagged > 500


def test_partitioned_edges(ctx):
    rows = synth.generate(synth.with_noise(synth.station(n=500, seed=88), 80, 190))
    _compare(ctx, rows, 20, 4, fl.MINMAX, 89, 2, 2, 1, 20, 1000, label="more partitions than fingerprints")
    _compare(ctx, rows[:3], 20, 4, fl.MINMAX, 89, 0, 1, 1, 20, 2, label="three fingerprints")
    a, b = fl.make_hash(89, 40)
    with pytest.raises(fl.FastLshError) as e:
        ctx.search_partitioned(fl.to_device_rows(rows), 4096, 20, 4, fl.MINMAX, a, b, 5, 2, n_partitions=0)
    assert e.value.code == fl.E_INVALID
