#!/usr/bin/env python3
"""Writes station90d.json: the CPU oracle's complete result for the 90-day
station search (7,776,000 fingerprints, 4096-dim, 200 set bits, Markov 70 %,
2,000 repeating sources; data seed 102, hash seed 202; Min-Max t = 100,
r = 4, lag 5, at least 4 votes, occurrence filter 1 %).

Calls only ``synth`` (the seeded inputs) and ``oracle`` (the plain CPU
search).  The oracle counts votes in vote partitions (ranges of the smaller
id) to bound host memory; partitioning leaves the result unchanged.

Stored: every counter of the search, the number of output pairs per vote
count, and the SHA-256 of the sorted output, each pair as 9 little-endian
bytes (uint32 i, uint32 j, uint8 votes).  Run time: about 10 minutes on 8
cores, about 30 GB of host memory.
"""
import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import synth  # noqa: E402

DIM, T, R, L, V, NUM, DEN = 4096, 100, 4, 5, 4, 1, 100
DATA_SEED, HASH_SEED, PARTS = 102, 202, 8
PAIR = np.dtype([("i", "<u4"), ("j", "<u4"), ("v", "u1")])


def digest(i, j, v) -> str:
    rec = np.empty(len(i), dtype=PAIR)
    rec["i"], rec["j"], rec["v"] = i, j, v
    return hashlib.sha256(rec.tobytes()).hexdigest()


def main():
    t0 = time.time()
    spec = synth.station(n=synth.STATION_90D, seed=DATA_SEED)
    rows = synth.generate(spec)
    print(f"generated {spec.n} rows in {time.time() - t0:.0f} s", flush=True)
    a, b = oracle.make_hash(HASH_SEED, oracle.n_funcs(T, R, oracle.MINMAX))
    keys = oracle.signatures(rows, DIM, T, R, oracle.MINMAX, a, b)
    del rows
    print(f"signatures done at {time.time() - t0:.0f} s", flush=True)
    oi, oj, ov, st = oracle.search_keys(keys, L, V, NUM, DEN, parts=PARTS)
    print(f"search done at {time.time() - t0:.0f} s: {st}", flush=True)
    hist = np.bincount(ov, minlength=T + 1)
    out = {
        "workload": "one station, 90 days at 1 s lag: 7,776,000 fingerprints, 4096-dim, 200 set bits, "
                    "Markov 70 %, 2,000 repeating sources (data seed 102); Min-Max t=100 r=4 (hash seed 202), "
                    "lag 5, v=4, occurrence filter 1/100",
        "n": spec.n, "dim": DIM, "tables": T, "rows": R, "scheme": "minmax", "min_lag": L, "min_votes": V,
        "occ_num": NUM, "occ_den": DEN, "data_seed": DATA_SEED, "hash_seed": HASH_SEED,
        "stats": st.__dict__,
        "pairs_by_votes": {str(k): int(c) for k, c in enumerate(hist) if c},
        "sha256_pairs": digest(oi, oj, ov),
        "pair_encoding": "sorted by (i, j); per pair uint32 i, uint32 j, uint8 votes, little-endian, packed",
        "written_by": "tests/golden/make_station90d.py (oracle and synth only)",
        "oracle_threads": oracle.max_threads(),
        "oracle_seconds": round(time.time() - t0, 1),
    }
    with open(os.path.join(HERE, "station90d.json"), "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")
    print(json.dumps(out["stats"]), out["sha256_pairs"], flush=True)


if __name__ == "__main__":
    main()
