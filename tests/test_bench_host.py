"""Host logic of bench.py, no GPU: the one-GPU rule, the source-hash gate on
the committed HBM traffic figures, and the roofline arithmetic of the line."""
import hashlib
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    # refused before anything touches a GPU or builds a workload
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert line["n_gpus"] == 2 and "one GPU" in line["error"]


def _traffic_tree(tmp_path, body=b"kernel body", n=1000):
    csrc = tmp_path / "paper_1803_09835_amd" / "csrc"
    csrc.mkdir(parents=True)
    (csrc / "k.hip").write_bytes(body)
    (csrc / "k.hpp").write_bytes(b"shared header")
    sha = hashlib.sha256(body + b"shared header").hexdigest()
    prof = tmp_path / "profiles"
    prof.mkdir()
    (prof / "k_one_traffic.txt").write_text(
        "# a comment line, with = in it, is skipped\n"
        f"kernel=k<1>\nn={n}\nsources=k.hip,k.hpp\nsource_sha256={sha}\nfetch_bytes=3000\nwrite_bytes=45\n")
    return csrc


def test_traffic_reported_only_for_its_size_and_sources(tmp_path, monkeypatch):
    csrc = _traffic_tree(tmp_path)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.kernel_traffic("k_one", 1000) == 3045
    assert bench.kernel_traffic("k_one", 999) is None          # taken at another size
    assert bench.kernel_traffic("k_missing", 1000) is None     # never taken
    (csrc / "k.hpp").write_bytes(b"shared header, changed")    # the kernel's code moved on
    assert bench.kernel_traffic("k_one", 1000) is None


def test_committed_traffic_files_are_complete():
    prof = os.path.join(ROOT, "profiles")
    files = [f for f in os.listdir(prof) if f.endswith("_traffic.txt")]
    assert files
    for f in files:
        kv = dict(l.strip().split("=", 1) for l in open(os.path.join(prof, f)) if "=" in l and not l.startswith("#"))
        assert {"kernel", "n", "sources", "source_sha256", "fetch_bytes", "write_bytes"} <= set(kv), f
        assert int(kv["n"]) > 0 and int(kv["fetch_bytes"]) > 0 and int(kv["write_bytes"]) >= 0, f
        assert len(kv["source_sha256"]) == 64, f
        for s in kv["sources"].split(","):
            assert os.path.exists(os.path.join(ROOT, "paper_1803_09835_amd", "csrc", s)), (f, s)


def test_tile_roofline_arithmetic():
    # 8 B per voted pair and 4 B per member over the kernel time per search
    work = {"big_voted": 10**12, "big_members": 5 * 10**9, "big_candidates": 10**12 + 7}
    r = bench.tile_roofline(work, None, 1000.0, 50)
    algo = 8 * 10**12 + 4 * 5 * 10**9
    assert r["algorithmic_bytes_per_search"] == algo
    assert r["achieved"] == round(algo / 1e9, 1)
    assert r["frac"] == round(algo / 1e9 / 8000.0, 4)
    assert r["peak"] == 8000.0 and r["bound"] == "hbm" and r["unit"] == "GB/s"
    assert r["launch_ms"] == 20.0 and r["launches_per_search"] == 50
    assert r["candidate_pairs_per_s"] == float(10**12 + 7)


def test_sig_roofline_arithmetic():
    # N x F x 200 evaluations at 3 int32 operations each (Min-Max), 2.5 (MinHash)
    assert round(bench.INT_PEAK_TOPS, 2) == 39.32  # 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz
    for scheme, ops in ((1, 3.0), (0, 2.5)):
        r = bench.sig_roofline(1000, 20, scheme, 2.0, 4, "k_sig")
        evals = 1000 * 20 * 200
        assert r["evals_per_s"] == round(evals / 0.002, 1)
        assert r["achieved"] == round(evals * ops / 0.002 / 1e12, 2)
        assert r["frac"] == round(evals * ops / 0.002 / 1e12 / bench.INT_PEAK_TOPS, 4)
        assert r["launch_ms"] == 0.5 and r["bound"] == "alu"
