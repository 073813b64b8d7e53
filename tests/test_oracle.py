"""Pins for the CPU oracle (runs without a GPU).

Nothing here retypes the oracle's formulas.  Each test checks the oracle
against something fixed independently: a published known answer, a special
case that reduces to a textbook quantity, an invariant of the mathematics,
a closed-form probability from the paper (section 6.3) or a brute force that
takes a different route (tests/brute.py).
"""
import math

import numpy as np
import pytest

import oracle
import synth
from tests import brute

P = oracle.P


# ---------------------------------------------------------------------------
# splitmix64 and the hash family
# ---------------------------------------------------------------------------
def test_splitmix64_published_values():
    # Known answers of splitmix64 for seed 0 (Steele, Lea & Flood 2014 reference generator).
    got = [int(x) for x in oracle.splitmix64_stream(0, 3)]
    assert got == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]


def test_make_hash_known_answer():
    # Function f draws a from output 2f and b from output 2f+1 of splitmix64
    # seeded with the seed.  Seed 0's outputs (the published reference
    # generator): 0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F,
    # 0xF88BB8A8724C81EC.  Worked out by hand:
    #   a[0] = 1 + 0xE220A8397B1DCDAF mod (2^31 - 2) = 60845732
    #   b[0] =     0x6E789E6AA1B965F4 mod (2^31 - 1) = 2125112010
    #   a[1] = 1 + 0x06C45D188009454F mod (2^31 - 2) = 454736306
    #   b[1] =     0xF88BB8A8724C81EC mod (2^31 - 1) = 1667494720
    # A swapped draw order, a wrong modulus or a missing "+1" changes them.
    out = [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F, 0xF88BB8A8724C81EC]
    assert [1 + out[0] % (P - 1), out[1] % P, 1 + out[2] % (P - 1), out[3] % P] == \
        [60845732, 2125112010, 454736306, 1667494720]
    assert [int(x) for x in oracle.splitmix64_stream(0, 4)] == out
    a, b = oracle.make_hash(0, 2)
    assert [int(x) for x in a] == [60845732, 454736306]
    assert [int(x) for x in b] == [2125112010, 1667494720]
    # Prefix property: the first functions do not depend on how many are drawn.
    a5, b5 = oracle.make_hash(0, 5)
    assert (a5[:2] == a).all() and (b5[:2] == b).all()


def test_make_hash_ranges_and_determinism():
    a, b = oracle.make_hash(202, 5000)
    assert a.min() >= 1 and a.max() <= P - 1
    assert b.max() <= P - 1
    a2, b2 = oracle.make_hash(202, 5000)
    assert (a == a2).all() and (b == b2).all()
    a3, _ = oracle.make_hash(203, 5000)
    assert (a != a3).mean() > 0.99
    # Parameters are spread over the whole range (uniform on [1, p-1]).
    assert 0.45 < a.mean() / P < 0.55


def test_hash_special_cases():
    # a = 1, b = 0 is the identity; a = p - 1 = -1 (mod p) is negation.
    for x in (0, 1, 7, 4095, 65535):
        assert oracle.hash_value(1, 0, x) == x
        assert oracle.hash_value(P - 1, 0, x) == (0 if x == 0 else P - x)
        assert oracle.hash_value(1, P - 1, x) == (x + P - 1) % P
    assert oracle.hash_value(P - 1, P - 1, 65535) == P - 1 - 65535


def test_hash_linearity_and_injectivity():
    rng = np.random.default_rng(1)
    for _ in range(200):
        a = int(rng.integers(1, P))
        b = int(rng.integers(0, P))
        x, y = (int(v) for v in rng.integers(0, 32768, 2))
        # h(x; a, 0) is a group homomorphism of Z_p: h(x + y) = h(x) + h(y).
        hx, hy, hxy = (oracle.hash_value(a, 0, v) for v in (x, y, x + y))
        assert hxy == (hx + hy) % P
        # Adding b shifts every value by b.
        assert oracle.hash_value(a, b, x) == (hx + b) % P
    # Injective on [0, d): a != 0 (mod p) and d < p.
    a, b = oracle.make_hash(9, 4)
    for f in range(4):
        vals = {oracle.hash_value(int(a[f]), int(b[f]), x) for x in range(4096)}
        assert len(vals) == 4096


# ---------------------------------------------------------------------------
# Signatures and band keys
# ---------------------------------------------------------------------------
def _fixed(n_rows, dim, nnz, seed):
    rng = np.random.default_rng(seed)
    return np.stack([np.sort(rng.choice(dim, nnz, replace=False)) for _ in range(n_rows)]).astype(np.uint16)


def test_identity_hash_gives_set_min_and_max():
    # With h(x) = x every MinHash value is min(S) and Min-Max gives (min S, max S).
    rows = _fixed(30, 4096, 37, 2)
    t, r = 3, 4
    a = np.ones(t * r, np.uint32)
    b = np.zeros(t * r, np.uint32)
    keys, vals = oracle.signatures(rows, 4096, t, r, oracle.MINHASH, a, b, with_values=True)
    assert (vals == rows.min(axis=1)[:, None, None]).all()
    keys, vals = oracle.signatures(rows, 4096, t, r, oracle.MINMAX, a, b, with_values=True)
    assert (vals[:, :, 0::2] == rows.min(axis=1)[:, None, None]).all()
    assert (vals[:, :, 1::2] == rows.max(axis=1)[:, None, None]).all()
    # Key = the attaining indices packed 12 bits apart: (min, max, min, max).
    lo = rows.min(axis=1).astype(np.uint64)
    hi = rows.max(axis=1).astype(np.uint64)
    expect = lo | (hi << np.uint64(12)) | (lo << np.uint64(24)) | (hi << np.uint64(36))
    assert (keys == expect[None, :]).all()


def test_negation_hash():
    # h(x) = -x mod p: the minimum is 0 if 0 is in the set, else p - max(S).
    rows = _fixed(40, 64, 5, 3)
    rows[0] = [0, 3, 9, 20, 63]
    a = np.full(1, P - 1, np.uint32)
    b = np.zeros(1, np.uint32)
    _, vals = oracle.signatures(rows, 64, 1, 1, oracle.MINHASH, a, b, with_values=True)
    for i, row in enumerate(rows):
        want = 0 if row.min() == 0 else P - int(row.max())
        assert vals[i, 0, 0] == want


def test_hand_worked_example():
    # d = 16 (4 key bits), Min-Max, one table with r = 4 rows, two functions:
    #   f0: h(x) = 3x + 5 (no wrap for x < 16, increasing)
    #   f1: h(x) = 7 - x mod p (decreasing, wraps for x > 7)
    # S = {2, 5, 11}:
    #   f0 values 11, 20, 38      -> min 11 at x=2,  max 38 at x=11
    #   f1 values 5, 2, p-4       -> min 2 at x=5,   max p-4 at x=11
    #   key = 2 | 11<<4 | 5<<8 | 11<<12 = 46514
    # S' = {2, 9, 11}: f0 -> (2, 11); f1 values 5, p-2, p-4 -> min 5 at x=2, max p-2 at x=9
    #   key = 2 | 11<<4 | 2<<8 | 9<<12 = 37554
    rows = np.array([[2, 5, 11], [2, 9, 11]], np.uint16)
    a = np.array([3, P - 1], np.uint32)
    b = np.array([5, 7], np.uint32)
    keys, vals = oracle.signatures(rows, 16, 1, 4, oracle.MINMAX, a, b, with_values=True)
    assert vals[0, 0].tolist() == [11, 38, 2, P - 4]
    assert vals[1, 0].tolist() == [11, 38, 5, P - 2]
    assert keys[0].tolist() == [46514, 37554]


@pytest.mark.parametrize("scheme,r", [(oracle.MINHASH, 4), (oracle.MINHASH, 3), (oracle.MINMAX, 4), (oracle.MINMAX, 2)])
@pytest.mark.parametrize("dim", [16, 1000, 4096])
def test_keys_match_brute_force(scheme, r, dim):
    rows = _fixed(25, dim, min(13, dim // 2), dim + r)
    t = 6
    nf = oracle.n_funcs(t, r, scheme)
    a, b = oracle.make_hash(dim * 7 + r, nf)
    keys = oracle.signatures(rows, dim, t, r, scheme, a, b)
    assert (keys == brute.keys_brute(rows, dim, t, r, scheme, a, b)).all()


def test_ragged_rows_match_fixed():
    rng = np.random.default_rng(4)
    lens = rng.integers(1, 30, 50)
    rows = [np.sort(rng.choice(512, L, replace=False)).astype(np.uint16) for L in lens]
    ind = np.concatenate(rows)
    off = np.concatenate([[0], np.cumsum(lens)]).astype(np.uint64)
    a, b = oracle.make_hash(5, 20)
    keys = oracle.signatures((ind, off), 512, 10, 4, oracle.MINMAX, a, b)
    assert (keys == brute.keys_brute(rows, 512, 10, 4, oracle.MINMAX, a, b)).all()


def test_band_key_decodes_to_attaining_elements():
    rows = _fixed(50, 4096, 200, 6)
    t, r = 5, 4
    a, b = oracle.make_hash(11, t * 2)
    keys, vals = oracle.signatures(rows, 4096, t, r, oracle.MINMAX, a, b, with_values=True)
    for i in range(len(rows)):
        S = set(rows[i].tolist())
        for u in range(t):
            k = int(keys[u, i])
            for s in range(r):
                x = (k >> (12 * s)) & 0xFFF
                f = u * 2 + s // 2
                assert x in S
                assert oracle.hash_value(int(a[f]), int(b[f]), x) == vals[i, u, s]


def test_invalid_inputs_rejected():
    a, b = oracle.make_hash(1, 8)
    with pytest.raises(ValueError):
        oracle.signatures(np.array([[3, 70]], np.uint16), 64, 2, 4, oracle.MINMAX, a, b)  # index >= d
    with pytest.raises(ValueError):
        oracle.signatures(np.array([[3, 3]], np.uint16), 64, 2, 4, oracle.MINMAX, a, b)   # duplicate
    with pytest.raises(ValueError):
        oracle.signatures(np.array([[3, 4]], np.uint16), 64, 2, 3, oracle.MINMAX, a, b)   # odd r, Min-Max
    with pytest.raises(ValueError):
        oracle.signatures((np.array([1], np.uint16), np.array([0, 0, 1], np.uint64)), 64, 2, 4,
                          oracle.MINMAX, a, b)                                             # empty row


# ---------------------------------------------------------------------------
# Probabilistic pins: section 6.1 (MinHash collision = Jaccard), the Min-Max
# collision law, and the banding S-curve of section 6.3.
# ---------------------------------------------------------------------------
def _pair_with_overlap(rng, dim, k, m):
    el = rng.choice(dim, 2 * k - m, replace=False)
    A = np.sort(el[:k])
    B = np.sort(np.concatenate([el[:m], el[k:2 * k - m]]))
    return np.stack([A, B]).astype(np.uint16)


# The linear family (a x + b) mod p restricted to [0, 4096) is only
# approximately min-wise independent (Broder et al. 1998).  Measured
# deviations from the ideal permutation law stay under 0.01 absolute; that is
# the extra slack delta below, on top of a 5-sigma binomial band.
DELTA = 0.01


@pytest.mark.parametrize("m", [40, 100, 160, 190])
def test_minhash_collision_probability_is_jaccard(m):
    rng = np.random.default_rng(m)
    F = 20000
    a, b = oracle.make_hash(1000 + m, F)
    pair = _pair_with_overlap(rng, 4096, 200, m)
    keys = oracle.signatures(pair, 4096, F, 1, oracle.MINHASH, a, b)
    J = m / (400 - m)
    est = (keys[:, 0] == keys[:, 1]).mean()
    assert abs(est - J) <= 5 * math.sqrt(J * (1 - J) / F) + DELTA


@pytest.mark.parametrize("m", [60, 150, 190])
def test_minmax_collision_law(m):
    # For a random permutation the (argmin, argmax) of A u B is a uniform
    # ordered pair of distinct elements, so both coincide for A and B with
    # probability m(m-1) / (n(n-1)), n = |A u B|.
    rng = np.random.default_rng(m + 1)
    F = 20000
    a, b = oracle.make_hash(2000 + m, F)
    pair = _pair_with_overlap(rng, 4096, 200, m)
    keys = oracle.signatures(pair, 4096, F, 2, oracle.MINMAX, a, b)
    n = 400 - m
    p = m * (m - 1) / (n * (n - 1))
    est = (keys[:, 0] == keys[:, 1]).mean()
    assert abs(est - p) <= 5 * math.sqrt(p * (1 - p) / F) + DELTA


def _tail(t, p, v):
    """Section 6.3: probability of at least v matching tables out of t."""
    return 1.0 - sum(math.comb(t, i) * (p ** i) * ((1 - p) ** (t - i)) for i in range(v))


@pytest.mark.parametrize("scheme,m", [(oracle.MINHASH, 170), (oracle.MINHASH, 185), (oracle.MINMAX, 170)])
def test_banding_s_curve(scheme, m):
    rng = np.random.default_rng(7 + m + scheme)
    t, r, npairs = 20, 4, 400
    nf = oracle.n_funcs(t, r, scheme)
    n = 400 - m
    J = m / n
    p1 = J if scheme == oracle.MINHASH else m * (m - 1) / (n * (n - 1))
    rows_per_table = r if scheme == oracle.MINHASH else r // 2
    votes = []
    for q in range(npairs):
        a, b = oracle.make_hash(50_000 + q, nf)
        keys = oracle.signatures(_pair_with_overlap(rng, 4096, 200, m), 4096, t, r, scheme, a, b)
        votes.append(int((keys[:, 0] == keys[:, 1]).sum()))
    votes = np.array(votes)
    # Per-table collision probability p = p1^(rows per table) (r=4 MinHash: J^4).
    p_lo = max(p1 - DELTA, 0) ** rows_per_table
    p_hi = min(p1 + DELTA, 1) ** rows_per_table
    for v in (1, 2, 4, 8):
        emp = (votes >= v).mean()
        lo, hi = _tail(t, p_lo, v), _tail(t, p_hi, v)
        sig = 5 * math.sqrt(max(lo * (1 - lo), hi * (1 - hi), 1e-4) / npairs)
        assert lo - sig <= emp <= hi + sig, (v, emp, lo, hi)


def test_identical_and_disjoint_fingerprints():
    rows = _fixed(3, 4096, 200, 8)
    rows[1] = rows[0]
    # row 2 disjoint from row 0
    rng = np.random.default_rng(9)
    rest = np.setdiff1d(np.arange(4096), rows[0])
    rows[2] = np.sort(rng.choice(rest, 200, replace=False))
    for scheme in (oracle.MINHASH, oracle.MINMAX):
        a, b = oracle.make_hash(33, 400)
        keys = oracle.signatures(rows, 4096, 100, 4, scheme, a, b)
        assert oracle.pair_votes(keys, 0, 1) == 100
        # Equal values need the same element, which must lie in both sets.
        assert oracle.pair_votes(keys, 0, 2) == 0


# ---------------------------------------------------------------------------
# Search: buckets, occurrence filter, self-match exclusion, votes
# ---------------------------------------------------------------------------
def _brute_compare(keys, L, v, num=0, den=0):
    oi, oj, ov, st, flags = oracle.search_keys(keys, L, v, num, den, want_flags=True)
    out, bst, bflags = brute.search_brute(keys, L, v, num, den)
    assert list(zip(oi.tolist(), oj.tolist(), ov.tolist())) == out
    assert st.__dict__ == bst
    assert (flags.astype(bool) == bflags).all()
    return st


@pytest.mark.parametrize("L,v", [(5, 2), (1, 1), (0, 1), (30, 3)])
def test_search_matches_all_pairs_uniform(L, v):
    rows = synth.generate(synth.tiny_uniform(n=1200, seed=3))
    # Small dimension and few bits make buckets crowded.
    a, b = oracle.make_hash(21, 20 * 4)
    keys = oracle.signatures(rows, 4096, 20, 4, oracle.MINHASH, a, b)
    small = synth.generate(synth.Spec(n=1200, dim=64, nnz=4, seed=4, n_sources=20, rep_min=3, rep_max=3,
                                      plant_keep=3))
    keys2 = oracle.signatures(small, 64, 20, 2, oracle.MINHASH, a, b)
    _brute_compare(keys, L, v)
    st = _brute_compare(keys2, L, v)
    assert st.e_raw > 1000


@pytest.mark.parametrize("num,den", [(0, 0), (1, 100), (1, 20), (3, 1000)])
def test_search_matches_all_pairs_markov(num, den):
    rows = synth.generate(synth.station(n=1500, seed=5, sources_per_90d=100_000))
    a, b = oracle.make_hash(22, 30 * 2)
    keys = oracle.signatures(rows, 4096, 30, 4, oracle.MINMAX, a, b)
    _brute_compare(keys, 5, 4, num, den)
    small = synth.generate(synth.Spec(n=1500, dim=32, nnz=6, seed=6, markov_keep=4, n_sources=30,
                                      rep_min=3, rep_max=9, jac_lo_milli=400, jac_hi_milli=900))
    keys2 = oracle.signatures(small, 32, 30, 2, oracle.MINMAX, a, b)
    st = _brute_compare(keys2, 5, 4, num, den)
    if den and num * 50 <= den:
        assert st.n_flagged > 0


def test_lag_boundary_hand_built():
    # Fingerprints 0, 4 and 5 are identical; everything else is distinct.
    keys = np.arange(10 * 3, dtype=np.uint64).reshape(3, 10) + np.uint64(100)
    keys[:, 4] = keys[:, 0]
    keys[:, 5] = keys[:, 0]
    oi, oj, ov, st = oracle.search_keys(keys, 5, 1)
    # (0,4): lag 4 < 5 dropped; (0,5): lag 5 kept; (4,5): lag 1 dropped.
    assert list(zip(oi.tolist(), oj.tolist(), ov.tolist())) == [(0, 5, 3)]
    assert st.e_raw == 3 * 3 and st.e_voted == 3 and st.n_distinct == 1 and st.max_bucket == 3


def test_occurrence_filter_hand_built():
    # N = 200, table 0 holds one bucket of 3 fingerprints (3 > 1 % of 200)
    # and one of 2 (2 = 1 %, not above): only the three are excluded, and
    # they take part in no pair of any table.
    t, n = 2, 200
    keys = np.arange(t * n, dtype=np.uint64).reshape(t, n) * np.uint64(7)
    keys[0, [10, 50, 90]] = 1
    keys[0, [20, 60]] = 2
    keys[1, [10, 150]] = 3     # 10 is excluded, so (10, 150) never counts
    keys[1, [60, 120]] = 4
    oi, oj, ov, st, flags = oracle.search_keys(keys, 5, 1, 1, 100, want_flags=True)
    assert np.nonzero(flags)[0].tolist() == [10, 50, 90]
    assert list(zip(oi.tolist(), oj.tolist(), ov.tolist())) == [(20, 60, 1), (60, 120, 1)]
    assert st.n_flagged == 3 and st.e_raw == 3 + 1 + 1 + 1


def test_votes_equal_definition_on_outputs():
    rows = synth.generate(synth.tiny_uniform(n=3000, seed=8))
    a, b = oracle.make_hash(201, 80)
    keys = oracle.signatures(rows, 4096, 20, 4, oracle.MINHASH, a, b)
    oi, oj, ov, st = oracle.search_keys(keys, 5, 2)
    assert st.n_out == len(oi) > 0
    for i, j, v in zip(oi[:200], oj[:200], ov[:200]):
        assert oracle.pair_votes(keys, int(i), int(j)) == v >= 2 and j - i >= 5
    # Output is sorted by (i, j) and unique.
    code = oi.astype(np.uint64) << np.uint64(32) | oj.astype(np.uint64)
    assert (np.diff(code.astype(np.int64)) > 0).all()


# ---------------------------------------------------------------------------
# The chained band key (ceil(log2 d) * r > 64)
# ---------------------------------------------------------------------------
def _partition_equal(a_labels, b_labels):
    """The two labellings induce the same partition of the items."""
    na = len(np.unique(a_labels))
    nb = len(np.unique(b_labels))
    joint = len(np.unique(np.stack([a_labels, b_labels], axis=1), axis=0))
    return na == nb == joint


@pytest.mark.parametrize("dim,r", [(8192, 8), (4096, 6)])
def test_chained_key_equality_is_tuple_equality(dim, r):
    # Above 64 packed bits the key is a chain of 64-bit mixes of the indices.
    # Equal index tuples must give equal keys and distinct tuples distinct
    # keys (a 64-bit collision among 1.3e6 tuples has probability ~5e-8).
    # Near neighbours differ in one coordinate by one (a chain that skipped a
    # coordinate or ignored the last one would collide on them) and exact
    # duplicates are included.
    assert oracle.key_bits(dim) * r > 64
    rng = np.random.default_rng(dim + r)
    n = 1_000_000
    tup = rng.integers(0, dim, (n, r), dtype=np.uint32)
    k = 200_000
    src = rng.integers(0, n, k)
    pos = rng.integers(0, r, k)
    near = tup[src].copy()
    near[np.arange(k), pos] = (near[np.arange(k), pos] + 1) % dim
    first = tup[rng.integers(0, n, 50_000)].copy()  # differ only in the first or last coordinate
    first[:, 0] = (first[:, 0] + 7) % dim
    last = tup[rng.integers(0, n, 50_000)].copy()
    last[:, -1] = (last[:, -1] + 7) % dim
    dup = tup[rng.integers(0, n, 50_000)]
    allt = np.concatenate([tup, near, first, last, dup])
    keys = oracle.band_keys(allt, dim)
    _, tlab = np.unique(allt, axis=0, return_inverse=True)
    _, klab = np.unique(keys, return_inverse=True)
    assert _partition_equal(tlab.ravel(), klab.ravel())


def test_chained_key_on_planted_pairs():
    # Through the whole signature path with chained keys (d = 4096, r = 6,
    # 72 packed bits): for every pair of copies of one planted source and for
    # neighbouring fingerprints of a Markov slice, the keys of a table are
    # equal exactly when the six hash values are (the hash is injective on
    # [0, d), so equal values mean equal attaining indices).
    t, r, dim = 12, 6, 4096
    for scheme in (oracle.MINHASH, oracle.MINMAX):
        a, b = oracle.make_hash(77, oracle.n_funcs(t, r, scheme))
        rows, lab = synth.generate(synth.tiny_uniform(n=4000, seed=78), labels=True)
        mk = synth.generate(synth.station(n=1500, seed=79))
        for data, pairs in ((rows, None), (mk, None)):
            keys, vals = oracle.signatures(data, dim, t, r, scheme, a, b, with_values=True)
            if data is rows:
                pairs = [(i, j) for src in np.unique(lab[lab >= 0])
                         for q, i in enumerate(np.nonzero(lab == src)[0]) for j in np.nonzero(lab == src)[0][q + 1:]]
            else:
                pairs = [(i, i + d) for i in range(len(data) - 3) for d in (1, 2, 3)]
            n_equal = 0
            for i, j in pairs:
                same_vals = (vals[i] == vals[j]).all(axis=1)
                same_keys = keys[:, i] == keys[:, j]
                assert (same_vals == same_keys).all()
                n_equal += int(same_keys.sum())
            assert n_equal > 0  # the planted and neighbouring pairs do share tables


def test_packed_key_used_up_to_64_bits():
    # ceil(log2 d) * r <= 64: the key is the packed indices, row s at bit b*s
    # (64 bits exactly at d = 65536, r = 4; 60 bits at d = 4096, r = 5).
    # One bit more (d = 4096, r = 6) switches to the chain.
    rng = np.random.default_rng(5)
    for dim, r in ((65536, 4), (4096, 5), (2, 64)):
        b = oracle.key_bits(dim)
        assert b * r <= 64
        tup = rng.integers(0, dim, (1000, r), dtype=np.uint64)
        want = np.zeros(1000, np.uint64)
        for s_ in range(r):
            want |= tup[:, s_] << np.uint64(b * s_)
        assert (oracle.band_keys(tup.astype(np.uint32), dim) == want).all()
    tup = rng.integers(0, 4096, (1000, 6), dtype=np.uint64)
    packed_low = np.zeros(1000, np.uint64)
    for s_ in range(5):
        packed_low |= tup[:, s_] << np.uint64(12 * s_)
    assert (oracle.band_keys(tup.astype(np.uint32), 4096) != packed_low).mean() > 0.99


# ---------------------------------------------------------------------------
# Vote partitions and the table-at-a-time form (used for full-size expected
# values) against the whole search, which the brute force pins
# ---------------------------------------------------------------------------
def _noise_keys(seed):
    rows = synth.generate(synth.with_noise(synth.station(n=6000, seed=seed), 40, 190))
    a, b = oracle.make_hash(seed + 1, 200)
    return oracle.signatures(rows, 4096, 100, 4, oracle.MINMAX, a, b)


def test_vote_partitions_change_nothing():
    # Counting the pairs one range of i at a time (section 6.4: partitioned
    # search gives the same result) concatenates to the same output.
    keys = _noise_keys(300)
    for num, den in ((0, 0), (1, 100)):
        whole = oracle.search_keys(keys, 5, 4, num, den)
        if den:
            assert whole[3].n_flagged > 0
        for parts in (2, 3, 7):
            got = oracle.search_keys(keys, 5, 4, num, den, parts=parts)
            for x, y in zip(whole[:3], got[:3]):
                assert np.array_equal(x, y)
            assert whole[3] == got[3]


def test_table_scan_matches_whole_search():
    # One table at a time, exclusions applied when the votes are counted:
    # identical to the whole search (every range of i), and restricted to the
    # ranges asked for otherwise; e_raw, max_bucket and n_flagged are global.
    keys = _noise_keys(310)
    t, n = keys.shape
    for num, den in ((0, 0), (1, 100)):
        ei, ej, ev, est = oracle.search_keys(keys, 5, 4, num, den)
        for ranges in ([(0, n)], [(0, 700), (2500, 2600), (5900, n)]):
            sc = oracle.TableScan(n, num, den, 5, ranges)
            for u in range(t):
                sc.add_table(keys[u])
            gi, gj, gv, gst = sc.result(4)
            sc.close()
            keep = np.zeros(len(ei), bool)
            for lo, hi in ranges:
                keep |= (ei >= lo) & (ei < hi)
            assert np.array_equal(gi, ei[keep]) and np.array_equal(gj, ej[keep]) and np.array_equal(gv, ev[keep])
            assert (gst.e_raw, gst.max_bucket, gst.n_flagged) == (est.e_raw, est.max_bucket, est.n_flagged)
            if ranges == [(0, n)]:
                assert gst == est
