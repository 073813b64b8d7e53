#!/usr/bin/env python3
"""Writes station5y_counters.json: the CPU oracle's exact global counters of
the 5-year station search (157,788,000 fingerprints, Markov 70 % in chains of
1,000,000, 20,000 repeating sources; data seed 105, hash seed 205; Min-Max
t = 100, r = 4, occurrence filter 1 %): e_raw (the raw candidate pairs summed
over tables), max_bucket and n_flagged.  Their definition needs only each
table's bucket sizes, so the oracle takes the tables a few at a time: for
every group the fingerprints are generated again slice by slice and the
group's band keys computed (the oracle's signatures with that group's hash
functions), then each table is sorted and its buckets counted.

Calls only ``synth`` and ``oracle``.  Run time: about 3.8 hours on six
threads of an 8-core machine, under 25 GB of host memory.
"""
import json
import os
import sys
import time
from concurrent.futures import ThreadPoolExecutor

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import synth  # noqa: E402

DIM, T, R, NUM, DEN = 4096, 100, 4, 1, 100
DATA_SEED, HASH_SEED, GROUP, SLICE = 105, 205, 4, 8_000_000


def main():
    t0 = time.time()
    spec = synth.long_station(n=synth.STATION_5Y, seed=DATA_SEED)
    n = spec.n
    a, b = oracle.make_hash(HASH_SEED, oracle.n_funcs(T, R, oracle.MINMAX))
    per = R // 2  # functions per table (Min-Max)
    e_raw, max_bucket = 0, 0
    flags = np.zeros(n, dtype=np.uint8)
    for g0 in range(0, T, GROUP):
        tabs = list(range(g0, min(T, g0 + GROUP)))
        fa = np.concatenate([a[u * per:(u + 1) * per] for u in tabs])
        fb = np.concatenate([b[u * per:(u + 1) * per] for u in tabs])
        keys = np.empty((len(tabs), n), dtype=np.uint64)
        for lo in range(0, n, SLICE):
            hi = min(n, lo + SLICE)
            rows = synth.generate(spec, lo, hi)
            keys[:, lo:hi] = oracle.signatures(rows, DIM, len(tabs), R, oracle.MINMAX, fa, fb)
        print(f"tables {tabs[0]}-{tabs[-1]}: keys at {time.time() - t0:.0f} s", flush=True)

        def scan(k):
            ts = oracle.TableScan(n, NUM, DEN, 0, [])
            ts.add_table(keys[k])
            return ts

        with ThreadPoolExecutor(len(tabs)) as ex:
            scans = list(ex.map(scan, range(len(tabs))))
        for ts in scans:
            e_raw += int(ts.e_raw.value)
            max_bucket = max(max_bucket, int(ts.max_bucket.value))
            flags |= ts.flags[:n]
            ts.close()
        del keys, scans
        print(f"tables {tabs[0]}-{tabs[-1]}: done at {time.time() - t0:.0f} s, e_raw so far {e_raw}", flush=True)
    out = {
        "workload": "one station, 5 years at 1 s lag: 157,788,000 fingerprints, 4096-dim, 200 set bits, Markov 70 % "
                    "in chains of 1,000,000, 20,000 repeating sources (data seed 105); Min-Max t=100 r=4 (hash seed "
                    "205), occurrence filter 1/100",
        "n": n, "tables": T, "rows": R, "occ_num": NUM, "occ_den": DEN, "data_seed": DATA_SEED,
        "hash_seed": HASH_SEED,
        "counters": {"e_raw": e_raw, "max_bucket": max_bucket, "n_flagged": int(flags.sum())},
        "written_by": "tests/golden/make_station5y_counters.py (oracle and synth only)",
        "oracle_threads": oracle.max_threads(), "oracle_seconds": round(time.time() - t0, 1),
    }
    with open(os.path.join(HERE, "station5y_counters.json"), "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")
    print(json.dumps(out["counters"]), flush=True)


if __name__ == "__main__":
    main()
