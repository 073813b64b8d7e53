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
