"""Host-side checks of the C-ABI library that need no GPU."""
import os
import re
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fast_lsh.h")


def _declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"\b(fast_lsh_[a-z_0-9]+)\s*\(", text)))


def _lib_path():
    from paper_1803_09835_amd import fast_lsh
    if not os.path.exists(fast_lsh.LIB_PATH):
        from paper_1803_09835_amd import build
        build.build()
    return fast_lsh.LIB_PATH


def test_header_declares_entry_points():
    names = _declared()
    for must in ("fast_lsh_signatures", "fast_lsh_search", "fast_lsh_ctx_create", "fast_lsh_make_hash"):
        assert must in names


def test_library_exports_every_declared_symbol():
    path = _lib_path()
    out = subprocess.run(["nm", "-D", "--defined-only", path], capture_output=True, text=True, check=True).stdout
    exported = set(re.findall(r"\bT (fast_lsh_[a-z_0-9]+)$", out, re.M))
    missing = [n for n in _declared() if n not in exported]
    assert not missing, missing


def test_library_does_not_link_the_oracle():
    path = _lib_path()
    out = subprocess.run(["nm", "-D", path], capture_output=True, text=True, check=True).stdout
    assert "orc_" not in out
    ldd = subprocess.run(["ldd", path], capture_output=True, text=True).stdout
    assert "liboracle" not in ldd


def test_binding_fails_loudly_without_library(tmp_path, monkeypatch):
    from paper_1803_09835_amd import fast_lsh
    monkeypatch.setattr(fast_lsh, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(fast_lsh, "_LIB", None)
    with pytest.raises(fast_lsh.FastLshError):
        fast_lsh.library()


def test_header_declares_the_serving_and_bounded_calls():
    names = _declared()
    for must in ("fast_lsh_search_batched", "fast_lsh_search_bounded", "fast_lsh_server_create",
                 "fast_lsh_server_submit", "fast_lsh_server_poll", "fast_lsh_server_take", "fast_lsh_plan_batch"):
        assert must in names


def _plan_brute(stations, max_batch):
    """The batching rule written out: oldest first, a station's chunk only if
    no earlier chunk of that station waits, at most max_batch."""
    out = []
    for k, s in enumerate(stations):
        if len(out) == max_batch:
            break
        if s not in stations[:k]:
            out.append(k)
    return out


def test_plan_batch_rule():
    _lib_path()
    import paper_1803_09835_amd as fl
    assert fl.plan_batch([], 8) == []
    assert fl.plan_batch([3, 3, 3], 8) == [0]
    assert fl.plan_batch([0, 1, 0, 2, 1, 3], 8) == [0, 1, 3, 5]
    assert fl.plan_batch([0, 1, 2, 3, 4], 2) == [0, 1]
    rng = np.random.default_rng(7)
    for _ in range(300):
        n = int(rng.integers(0, 40))
        st = rng.integers(0, 6, n).tolist()
        mb = int(rng.integers(1, 10))
        got = fl.plan_batch(st, mb)
        assert got == _plan_brute(st, mb)
        # invariants: distinct stations, each the oldest waiting chunk of its station
        assert len({st[k] for k in got}) == len(got) and len(got) <= mb
