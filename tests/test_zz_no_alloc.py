"""The allocation-free channel merge (fast_lsh_channel_merge_noalloc, fixed
scratch array, no device allocation) against the allocating merge and the
oracle: two calls in a row on one context, the second with a smaller input,
then a call on a fresh context after other work, and an input beyond the
scratch limit (rejected on the host before any launch)."""
import sys

import numpy as np
import pytest

import oracle
from align_inputs import channels

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_1803_09835_amd as fl  # noqa: E402

MAX_PAIRS = 1_860_736  # the header's stated limit for 64 MiB of scratch


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _dev(chs):
    return [(torch.from_numpy(i.view(np.int32)).cuda(), torch.from_numpy(j.view(np.int32)).cuda(),
             torch.from_numpy(v).cuda()) for i, j, v in chs]


def _same(a, b):
    return all(torch.equal(x, y) for x, y in zip(a, b))


def test_noalloc_merge_matches_allocating_merge():
    ctx = fl.FastLSH(0)
    big = channels(31, 3, 5_000_000, 600_000, shared=0.3)        # 1.8 M pairs in all, close to the limit
    small = channels(32, 2, 20_000, 4_000, shared=0.5)
    say(f"[noalloc] call 1: {sum(len(c[0]) for c in big)} pairs; call 2: {sum(len(c[0]) for c in small)} pairs")
    for chs, n, min_sim in ((big, 5_000_000, 5), (small, 20_000, 3)):
        d = _dev(chs)
        got = ctx.channel_merge(d, n, min_sim, noalloc=True)
        ref = ctx.channel_merge(d, n, min_sim)
        assert _same(got, ref)
        want = oracle.channel_merge(chs, min_sim)
        assert all(np.array_equal(g.cpu().numpy().view(np.uint32), w) for g, w in zip(got, want))
        say(f"[noalloc] {len(want[0])} merged entries agree")
    ctx.close()
    # a second context on the same device shares the array; earlier contents do not matter
    ctx2 = fl.FastLSH(0)
    d = _dev(small)
    assert _same(ctx2.channel_merge(d, 20_000, 0, noalloc=True), ctx2.channel_merge(d, 20_000, 0))
    ctx2.close()


def test_noalloc_merge_limits():
    ctx = fl.FastLSH(0)
    n = MAX_PAIRS + 1
    i = torch.zeros(n, dtype=torch.int32, device="cuda")
    j = torch.ones(n, dtype=torch.int32, device="cuda")
    v = torch.ones(n, dtype=torch.uint8, device="cuda")
    with pytest.raises(fl.FastLshError) as e:
        ctx.channel_merge([(i, j, v)], 10, 0, noalloc=True)
    assert e.value.code == fl.E_NOMEM
    # exactly at the limit: one key repeated MAX_PAIRS times, summed once
    out = ctx.channel_merge([(i[:MAX_PAIRS], j[:MAX_PAIRS], v[:MAX_PAIRS])], 10, 0, noalloc=True)
    assert [int(x[0]) for x in out] == [1, 0, MAX_PAIRS] and out[0].numel() == 1
    # empty input and a bad pair behave as in the allocating merge
    assert [x.numel() for x in ctx.channel_merge([], 10, 0, noalloc=True)] == [0, 0, 0]
    with pytest.raises(fl.FastLshError) as e:
        ctx.channel_merge([(j[:2], i[:2], v[:2])], 10, 0, noalloc=True)
    assert e.value.code == fl.E_INVALID
    ctx.close()
