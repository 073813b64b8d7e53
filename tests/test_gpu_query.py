"""GPU parity of query-only hashing (section 6.4) through the C-ABI: the
(query, item, votes) output against the oracle element by element, and
against the cross pairs of a whole search of dataset plus queries."""
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


def _queries(data, nq, seed, dim=4096, nnz=200):
    """Queries: rows of the dataset (and their neighbours' structure) plus
    independent uniform rows."""
    rng = np.random.default_rng(seed)
    pick = rng.choice(len(data), nq // 2, replace=False)
    other = synth.generate(synth.Spec(n=nq - nq // 2, dim=dim, nnz=nnz, seed=seed))
    return np.concatenate([data[pick], other])


def _check(ctx, q, d, dim, t, r, scheme, seed, v, label):
    say(f"[query] {label}: {len(q)} queries, {len(d)} items, t={t} r={r} v={v}")
    a, b = fl.make_hash(seed, fl.n_funcs(t, r, scheme))
    gq, gx, gv, st = ctx.query(fl.to_device_rows(q), fl.to_device_rows(d), dim, t, r, scheme, a, b, v)
    wq, wx, wv, nc = oracle.query(q, d, dim, t, r, scheme, a, b, v)
    assert np.array_equal(_u32(gq), wq) and np.array_equal(_u32(gx), wx) and np.array_equal(gv.cpu().numpy(), wv)
    assert st.n_out == len(wq) and st.e_raw == nc
    return st


@pytest.mark.parametrize("nq,nd,t,r,scheme,v", [(500, 50_000, 100, 4, fl.MINMAX, 4), (200, 20_000, 20, 4,
                                                                                   fl.MINHASH, 2),
                                                (1, 10_000, 10, 2, fl.MINMAX, 1), (10_000, 100_000, 20, 4,
                                                                                   fl.MINHASH, 3)])
def test_query_matches_oracle(ctx, nq, nd, t, r, scheme, v):
    # 10,000 queries exceed the LDS stage (8,192 keys): bisection from HBM
    d = synth.generate(synth.station(n=nd, seed=71))
    q = _queries(d, nq, 72)
    st = _check(ctx, q, d, 4096, t, r, scheme, 73, v, f"{nq}x{nd}")
    assert st.n_out >= nq // 2


def test_query_chained_keys(ctx):
    # 8192-dim, r = 8: 104 key bits, the chained 64-bit key (all 64 bits sorted)
    rng = np.random.default_rng(5)
    d = np.array([np.sort(rng.choice(8192, 60, replace=False)) for _ in range(3000)], dtype=np.uint16)
    q = d[rng.choice(3000, 100, replace=False)].copy()
    q[::2, :10] = np.sort(rng.choice(8192, (50, 10)), axis=1)  # perturbed copies
    q = np.sort(q, axis=1)
    ok = np.array([len(np.unique(row)) == 60 for row in q])
    _check(ctx, q[ok], d, 8192, 30, 8, fl.MINMAX, 74, 2, "chained")


def test_query_equals_whole_search(ctx):
    # section 6.4: the same pairs as a search over tables holding everything
    d = synth.generate(synth.station(n=30_000, seed=75))
    q = _queries(d, 400, 76)
    a, b = fl.make_hash(77, fl.n_funcs(100, 4, fl.MINMAX))
    gq, gx, gv, _ = ctx.query(fl.to_device_rows(q), fl.to_device_rows(d), 4096, 100, 4, fl.MINMAX, a, b, 4)
    both = fl.to_device_rows(np.concatenate([d, q]))
    i, j, v, _ = ctx.search(both, 4096, 100, 4, fl.MINMAX, a, b, 1, 4)
    i, j, v = _u32(i), _u32(j), v.cpu().numpy()
    cross = (i < len(d)) & (j >= len(d))
    want = np.lexsort((i[cross], j[cross] - len(d)))
    assert np.array_equal(_u32(gq), (j[cross] - len(d))[want]) and np.array_equal(_u32(gx), i[cross][want])
    assert np.array_equal(gv.cpu().numpy(), v[cross][want])


def test_query_edges(ctx):
    d = synth.generate(synth.station(n=5000, seed=78))
    q = _queries(d, 50, 79)
    a, b = fl.make_hash(80, 200)
    empty = fl.to_device_rows(np.empty((0, 200), np.uint16))
    out = ctx.query(empty, fl.to_device_rows(d), 4096, 100, 4, fl.MINMAX, a, b, 1)
    assert out[3].n_out == 0
    out = ctx.query(fl.to_device_rows(q), empty, 4096, 100, 4, fl.MINMAX, a, b, 1)
    assert out[3].n_out == 0
    full = ctx.query(fl.to_device_rows(q), fl.to_device_rows(d), 4096, 100, 4, fl.MINMAX, a, b, 1)
    with pytest.raises(fl.FastLshError) as e:
        ctx.query(fl.to_device_rows(q), fl.to_device_rows(d), 4096, 100, 4, fl.MINMAX, a, b, 1,
                  capacity=full[3].n_out - 1)
    assert e.value.code == fl.E_CAPACITY
    bad = q.copy()
    bad[0, -1] = 4096  # index >= dim
    with pytest.raises(fl.FastLshError) as e:
        ctx.query(fl.to_device_rows(bad), fl.to_device_rows(d), 4096, 100, 4, fl.MINMAX, a, b, 1)
    assert e.value.code == fl.E_INVALID
