"""GPU parity of the spatiotemporal alignment (section 7) through the C-ABI:
the channel merge and the station clusters against the CPU oracle, element
by element (integers: exact), on seeded inputs and on the merged outputs of
three channels of one station searched on the GPU."""
import sys

import numpy as np
import pytest

import oracle
import synth
from align_inputs import channels, entries

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


def _dev(chs):
    return [(torch.from_numpy(i.view(np.int32)).cuda(), torch.from_numpy(j.view(np.int32)).cuda(),
             torch.from_numpy(v).cuda()) for i, j, v in chs]


def _u32(t):
    return t.cpu().numpy().view(np.uint32)


def _merge_both(ctx, chs, n, min_sim, label):
    say(f"[merge] {label}: {len(chs)} channels, {sum(len(c[0]) for c in chs)} pairs, n={n}, min_sim={min_sim}")
    g = ctx.channel_merge(_dev(chs), n, min_sim)
    w = oracle.channel_merge(chs, min_sim)
    for x, y in zip(g, w):
        assert np.array_equal(_u32(x), y)
    return w


@pytest.mark.parametrize("seed,n_ch,n,pairs,min_sim", [(1, 3, 400, 300, 0), (2, 3, 400, 300, 9),
                                                      (3, 1, 1000, 800, 1), (4, 5, 3000, 2000, 20),
                                                      (5, 3, 2_000_000, 400_000, 6),
                                                      (6, 3, 300_000_000, 1_000_000, 4)])
def test_channel_merge_matches_oracle(ctx, seed, n_ch, n, pairs, min_sim):
    # n = 3e8 uses 29-bit ids (four radix digits each for dt and idx1)
    _merge_both(ctx, channels(seed, n_ch, n, pairs, shared=0.3), n, min_sim, f"seed {seed}")


def test_channel_merge_edges(ctx):
    chs = channels(7, 3, 500, 200)
    empty = (np.empty(0, np.uint32), np.empty(0, np.uint32), np.empty(0, np.uint8))
    _merge_both(ctx, [empty, chs[0], empty, chs[1]], 500, 0, "empty channels")
    _merge_both(ctx, [empty], 500, 0, "only empty")
    assert [len(x) for x in ctx.channel_merge([], 500, 0)] == [0, 0, 0]
    # threshold above every sum: nothing survives
    w = _merge_both(ctx, chs, 500, 10_000, "all dropped")
    assert len(w[0]) == 0
    # capacity overflow reports the count and writes nothing
    m = len(oracle.channel_merge(chs, 0)[0])
    with pytest.raises(fl.FastLshError) as e:
        ctx.channel_merge(_dev(chs), 500, 0, capacity=m - 1)
    assert e.value.code == fl.E_CAPACITY
    # a pair with j <= i, or an id beyond n, is rejected
    bad = (np.array([5, 9], np.uint32), np.array([7, 9], np.uint32), np.array([1, 1], np.uint8))
    with pytest.raises(fl.FastLshError) as e:
        ctx.channel_merge(_dev([bad]), 500, 0)
    assert e.value.code == fl.E_INVALID
    with pytest.raises(fl.FastLshError) as e:
        ctx.channel_merge(_dev(chs), 400, 0)
    assert e.value.code == fl.E_INVALID


def _clusters_both(ctx, dt, idx1, sim, gap, width, me=1, ms=0, label=""):
    say(f"[clusters] {label}: {len(dt)} entries, gap {gap}, width {width}, min_entries {me}, min_sum {ms}")
    g = ctx.station_clusters(torch.from_numpy(dt.view(np.int32)).cuda(), torch.from_numpy(idx1.view(np.int32)).cuda(),
                             torch.from_numpy(sim.view(np.int32)).cuda(), gap, width, me, ms)
    got = g.cpu().numpy().view(fl.CLUSTER_DTYPE).reshape(-1)
    want = oracle.station_clusters(dt, idx1, sim, gap, width, me, ms)
    assert got.tobytes() == want.tobytes(), (len(got), len(want))
    return want


@pytest.mark.parametrize("seed,gap,width,me,ms", [(1, 1, 1, 1, 0), (2, 3, 2, 2, 0), (3, 5, 3, 3, 20),
                                                  (4, 10, 12, 1, 0), (5, 0, 5, 1, 0), (6, 4, 1, 5, 40)])
def test_station_clusters_small(ctx, seed, gap, width, me, ms):
    _clusters_both(ctx, *entries(seed), gap, width, me, ms, label=f"seed {seed}")


@pytest.mark.parametrize("seed,gap,width", [(11, 3, 3), (12, 20, 2), (13, 1, 100)])
def test_station_clusters_large(ctx, seed, gap, width):
    # many diagonals, long streaks spanning several waves, dense noise
    dt, idx1, sim = entries(seed, n_diag=5000, streaks=20000, noise=2_000_000, span=5_000_000,
                            streak_len=(10, 400), step=(1, 6))
    c = _clusters_both(ctx, dt, idx1, sim, gap, width, 3, 10, label=f"large seed {seed}")
    assert len(c) > 100


def test_station_clusters_one_long_run(ctx):
    # one diagonal of 1e6 consecutive entries: one run, one cluster
    n = 1_000_000
    dt = np.full(n, 5, np.uint32)
    idx1 = np.arange(n, dtype=np.uint32) * 2
    sim = (np.arange(n) % 7 + 1).astype(np.uint32)
    c = _clusters_both(ctx, dt, idx1, sim, 2, 1, label="one long run")
    assert len(c) == 1 and int(c[0]["n_entries"]) == n


def test_station_clusters_edges(ctx):
    dt, idx1, sim = entries(21)
    for k in (0, 1, 2):
        _clusters_both(ctx, dt[:k], idx1[:k], sim[:k], 3, 3, label=f"{k} entries")
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a).view(np.int32)).cuda()
    with pytest.raises(fl.FastLshError) as e:  # out of order
        ctx.station_clusters(t(dt[::-1]), t(idx1[::-1]), t(sim), 3, 3)
    assert e.value.code == fl.E_INVALID
    with pytest.raises(fl.FastLshError) as e:  # a repeated entry
        ctx.station_clusters(t(np.r_[dt[:1], dt[:1]]), t(np.r_[idx1[:1], idx1[:1]]), t(sim[:2]), 3, 3)
    assert e.value.code == fl.E_INVALID
    big = sim.copy()
    big[3] = 1 << 24
    with pytest.raises(fl.FastLshError) as e:
        ctx.station_clusters(t(dt), t(idx1), t(big), 3, 3)
    assert e.value.code == fl.E_INVALID
    m = len(oracle.station_clusters(dt, idx1, sim, 3, 3))
    with pytest.raises(fl.FastLshError) as e:
        ctx.station_clusters(t(dt), t(idx1), t(sim), 3, 3, capacity=m - 1)
    assert e.value.code == fl.E_CAPACITY


def test_three_channels_of_a_station(ctx):
    """Three channels of one station (shared planted sources, per-channel
    background and copies) searched on the GPU with a lenient threshold,
    merged and clustered on the GPU; the oracle does every step itself."""
    n, t, r, L, v = 120_000, 100, 4, 5, 2
    a, b = fl.make_hash(202, fl.n_funcs(t, r, fl.MINMAX))
    gpu_out, cpu_out = [], []
    for ch in range(3):
        rows = synth.generate(synth.Spec(n=n, seed=102, markov_keep=140, n_sources=60, rep_min=3, rep_max=40,
                                         jac_lo_milli=400, jac_hi_milli=900, channel=ch))
        gi, gj, gv, _ = ctx.search(fl.to_device_rows(rows), 4096, t, r, fl.MINMAX, a, b, L, v)
        gpu_out.append((gi, gj, gv))
        ei, ej, ev, _ = oracle.search(rows, 4096, t, r, oracle.MINMAX, a, b, L, v)
        cpu_out.append((ei, ej, ev))
        assert np.array_equal(_u32(gi), ei) and np.array_equal(_u32(gj), ej)
        say(f"[station] channel {ch}: {len(ei)} pairs")
    for min_sim in (6, 12):
        gdt, gx, gs = ctx.channel_merge(gpu_out, n, min_sim)
        wdt, wx, ws = oracle.channel_merge(cpu_out, min_sim)
        assert np.array_equal(_u32(gdt), wdt) and np.array_equal(_u32(gx), wx) and np.array_equal(_u32(gs), ws)
        say(f"[station] merged at {min_sim}: {len(wdt)} entries")
        g = ctx.station_clusters(gdt, gx, gs, 10, 3, 2, 0).cpu().numpy().view(fl.CLUSTER_DTYPE).reshape(-1)
        w = oracle.station_clusters(wdt, wx, ws, 10, 3, 2, 0)
        assert g.tobytes() == w.tobytes() and len(w) > 0
