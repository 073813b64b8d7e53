#!/usr/bin/env python3
"""Throughput and streaming latency of the LSH similarity search on one MI355X.

Default workload (the largest one-GPU configuration): one station, 5 years of
fingerprints at a 1 s lag (157,788,000 fingerprints, 4096-dim, 200 set bits
each; Markov background keeping 70 % of the previous fingerprint; 20,000
repeating sources with 3-40 copies whose Jaccard similarity to the template
is U[0.4, 0.9]).  Min-Max hash, t = 100 tables, r = 4 rows (2 functions per
table), self-match lag 5, at least 4 votes, occurrence filter at 1 % of N;
the tables are taken 10 at a time so that the search fits in HBM.

One step = one full search: signatures, grouping of all 100 tables, bucket
segmentation and occurrence filter, in-bucket pair votes, threshold and
canonical sort, from fingerprints resident in HBM to the sorted pairs in HBM
and the pair count on the host.  value = fingerprints / second.

After the timed steps the same process runs the streaming workload (8
stations of 180 days resident, 3,600-fingerprint chunks arriving as Poisson
streams at 40 chunks/s) and adds its p50/p99 chunk latency and sustained
chunk rate to the line, next to the time a plain search of one station's
history plus one chunk takes on the same GPU.

Other workloads (--workload):
  station       90 days, 7,776,000 fingerprints, tables all at once;
  bounded       the 5-year search alone;
  serving       the streaming workload alone;
  batched       12 stations in one search against 12 sequential searches;
  alignment     three channels of the 90-day station searched, then the
                channel merge and the station clusters;
  query         1,000 queries hashed against the 90-day station (query-only
                hashing) against the plain search of both;
  partitioned   the 90-day station in three 30-day partitions with the
                dynamic, per-partition occurrence filter;
  fingerprints  fingerprint extraction from 90 days of 100 Hz waveform.
Prints one JSON line.
"""
from __future__ import annotations

import argparse
import gc
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "fingerprints/s through MinHash+LSH vote count; p50/p99 streaming chunk latency"

# MI355X published peaks and unit counts
HBM_PEAK_GBS = 8000.0
CUS, SIMDS_PER_CU, LANES_PER_SIMD, CLOCK_GHZ = 256, 4, 16, 2.4
INT_PEAK_TOPS = CUS * SIMDS_PER_CU * LANES_PER_SIMD * CLOCK_GHZ / 1000.0  # 39.32 T int32 lane-ops/s

# Algorithmic int32 operations per hash evaluation h(x) = (a x + b) mod (2^31-1)
# with its extreme updates: one 32x32->64-bit multiply-add and one shift-add
# for the Mersenne fold (twice the folded value, 2 (y mod 2^31) + 2 (y >> 31)
# wrapped to 32 bits, kept in order), then the extreme updates with
# three-input min/max, which fold two new values per instruction: 1/2 per
# tracked extreme (min for MinHash; min and max for Min-Max).  The folded value
# is the hash value whenever it is below p, which the kernel checks with the
# running extremes (for MinHash the maximum, an extra half operation that is
# not counted, like the half operation that unpacks two 16-bit indices per
# register).
OPS_PER_EVAL = {0: 2.5, 1: 3.0}  # MinHash, Min-Max

# Algorithmic bytes of the pair stages: one 8-byte vote update per valid
# candidate pair (a pair passing the lag and the exclusion, counted in
# e_voted) and one 4-byte id read per bucket member.
BYTES_PER_VOTED_PAIR, BYTES_PER_MEMBER = 8, 4


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def kernel_traffic(name, n):
    """HBM bytes per launch of a kernel from the committed counter figures
    (profiles/<name>_traffic.txt), or None when they were taken for another
    size or on different kernel code (the file holds the SHA-256 of the
    sources it lists)."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"{name}_traffic.txt")
    if not os.path.exists(path):
        return None
    kv = dict(l.strip().split("=", 1) for l in open(path) if "=" in l and not l.startswith("#"))
    files = kv.get("sources", "sig.hip,common.hpp").split(",")
    src = b"".join(open(os.path.join(ROOT, "paper_1803_09835_amd", "csrc", f), "rb").read() for f in files)
    if int(kv.get("n", -1)) != n or kv.get("source_sha256") != hashlib.sha256(src).hexdigest():
        return None
    return int(kv["fetch_bytes"]) + int(kv["write_bytes"])


def parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--workload", choices=("headline", "station", "batched", "bounded", "serving", "alignment",
                                           "query", "partitioned", "fingerprints"),
                    default="headline",
                    help="headline (default): the 5-year station (157,788,000 fingerprints, tables 10 at a "
                         "time) timed over the steps, then the streaming workload's latency; station: one "
                         "90-day station; bounded: the 5-year search alone; serving: 8 stations of 180 days "
                         "resident, 3,600-row chunks arriving as Poisson streams; batched: 12 stations of "
                         "1-16 M fingerprints in one search, against 12 sequential searches; alignment: three "
                         "channels of the 90-day station searched with a lenient threshold, then their channel "
                         "merge and station clusters timed; query: 1,000 queries against the 90-day station "
                         "with only the queries hashed, beside the plain search of both; partitioned: the "
                         "90-day station in three partitions with the dynamic occurrence filter; fingerprints: "
                         "fingerprint extraction of 90 days of 100 Hz waveform (7,776,000 fingerprints)")
    ap.add_argument("--chunks", type=int, default=3000, help="serving: chunks at the offered load")
    ap.add_argument("--rate", type=float, default=40.0, help="serving: offered chunks/s (all stations)")
    ap.add_argument("--stations", type=int, default=8, help="serving: stations")
    ap.add_argument("--group-tables", type=int, default=10, help="bounded: tables per group")
    ap.add_argument("--graph", action="store_true", help="replay the captured graph of the search prefix")
    ap.add_argument("--autotune", action="store_true", help="tune launch shapes on the first (warm-up) search")
    ap.add_argument("--bin-bits", type=int, default=0,
                    help="key bits the grouping passes sort on (8/16/24/32; 0: automatic)")
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=0, help="fingerprints (0: the workload's own size)")
    ap.add_argument("--cpu-sample", type=int, default=1_000_000,
                    help="fingerprints of the same workload the CPU oracle is timed on, all threads (0: skip)")
    ap.add_argument("--cpu-sample-1t", type=int, default=100_000,
                    help="fingerprints the CPU oracle is timed on with one thread (0: skip)")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="after timing, copy this many MiB device-to-device with a plain copy kernel "
                         "(reference dispatch for HBM counter calibration)")
    return ap.parse_args()


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU: no search, batch or server is sharded over "
                                   "several GPUs", "n_gpus": args.gpus}))
        sys.exit(2)
    if args.workload == "headline":
        line = run_bounded(args)
        free_gpu()
        srv, spec0 = run_serving(args)
        free_gpu()
        plain = run_plain_chunk(spec0)
        free_gpu()
        line["metric"] = METRIC
        line["latency_ms"] = srv["offered_load"]["latency_ms"]
        srv["plain_search_of_history_plus_chunk"] = plain
        line["serving"] = srv
    elif args.workload == "station":
        line = run_station(args)
    elif args.workload == "bounded":
        line = run_bounded(args)
    elif args.workload == "serving":
        line, _ = run_serving(args)
        line["metric"] = METRIC
        line["latency_ms"] = line["offered_load"]["latency_ms"]
    elif args.workload == "alignment":
        line = run_alignment(args)
    elif args.workload == "query":
        line = run_query(args)
    elif args.workload == "partitioned":
        line = run_partitioned(args)
    elif args.workload == "fingerprints":
        line = run_fingerprints(args)
    else:
        line = run_batched(args)
    print(json.dumps(line), flush=True)


def free_gpu():
    import torch
    gc.collect()
    torch.cuda.synchronize()
    torch.cuda.empty_cache()


def time_oracle(rows, dim, t, r, scheme, a, b, L, v, occ_num, occ_den, threads=0):
    import oracle
    if threads:
        oracle.set_threads(threads)
    used = oracle.max_threads()
    tc = time.perf_counter()
    oracle.search(rows, dim, t, r, scheme, a, b, L, v, occ_num, occ_den)
    return time.perf_counter() - tc, used


def cpu_baseline(rows_of, dim, t, r, scheme, a, b, L, v, occ_num, occ_den, args, label):
    """The oracle timed on the host on the first fingerprints of the workload:
    all threads on --cpu-sample rows, one thread on --cpu-sample-1t rows."""
    import oracle
    out = None
    all_threads = oracle.max_threads()
    if args.cpu_sample > 0:
        rows = rows_of(args.cpu_sample)
        s, used = time_oracle(rows, dim, t, r, scheme, a, b, L, v, occ_num, occ_den)
        out = {"value": round(len(rows) / s, 1), "unit": "fingerprints/s", "cores": used, "kind": "oracle",
               "cpu": cpu_model(),
               "sample": f"first {len(rows)} fingerprints of {label}, searched alone (signatures + votes) in "
                         f"{s:.1f} s on {used} threads; the pair work grows faster than N, so a slice "
                         f"over-states the CPU rate at full size"}
        log(f"# cpu oracle: {len(rows)} rows in {s:.1f} s on {used} threads")
    if args.cpu_sample_1t > 0:
        rows = rows_of(args.cpu_sample_1t)
        s, used = time_oracle(rows, dim, t, r, scheme, a, b, L, v, occ_num, occ_den, threads=1)
        oracle.set_threads(all_threads)
        one = {"value": round(len(rows) / s, 1), "unit": "fingerprints/s", "cores": used,
               "sample": f"first {len(rows)} fingerprints, {s:.1f} s on one thread"}
        log(f"# cpu oracle: {len(rows)} rows in {s:.1f} s on 1 thread")
        if out is None:
            out = dict(one, kind="oracle", cpu=cpu_model())
        else:
            out["single_thread"] = one
    return out


def stage_table(prof, steps):
    return ({k: ms / steps for k, (ms, n) in prof.items()}, {k: n / steps for k, (ms, n) in prof.items()})


def sig_roofline(N, nf, scheme, sig_ms, launches, kernel):
    """k_sig against the int32 VALU peak: N x F x 200 evaluations per search."""
    evals = N * nf * 200
    achieved = evals * OPS_PER_EVAL[scheme] / (sig_ms / 1000.0) / 1e12
    return {"kernel": kernel, "bound": "alu", "achieved": round(achieved, 2), "peak": round(INT_PEAK_TOPS, 2),
            "unit": "TOP/s (int32)", "frac": round(achieved / INT_PEAK_TOPS, 4),
            "evals_per_s": round(evals / (sig_ms / 1000.0), 1),
            "launch_ms": round(sig_ms / max(launches, 1), 3), "launches_per_search": launches}


def tile_roofline(work, st, tile_ms, launches):
    """k_pairs_tile against HBM: 8 B per valid candidate pair it counts and 4 B
    per member of the buckets it takes, over its kernel time per search."""
    algo = BYTES_PER_VOTED_PAIR * work["big_voted"] + BYTES_PER_MEMBER * work["big_members"]
    gbs = algo / (tile_ms / 1000.0) / 1e9
    return {"kernel": "k_pairs_tile<17,true,true>", "bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": None,
            "algorithmic_bytes_per_search": algo,
            "units": {"voted_pairs": work["big_voted"], "members": work["big_members"],
                      "candidate_pairs": work["big_candidates"]},
            "candidate_pairs_per_s": round(work["big_candidates"] / (tile_ms / 1000.0), 1),
            "launch_ms": round(tile_ms / max(launches, 1), 3), "launches_per_search": launches,
            "kernel_ms_per_search": round(tile_ms, 3)}


def run_station(args):
    """One 90-day station, every table at once."""
    import torch

    import synth
    import paper_1803_09835_amd as fl

    N = args.n or synth.STATION_90D
    dim, t, r, scheme = 4096, 100, 4, fl.MINMAX
    L, v, occ_num, occ_den = 5, 4, 1, 100
    spec = synth.station(n=N, seed=102)
    tg = time.time()
    rows = synth.generate(spec)
    gen_s = time.time() - tg
    a, b = fl.make_hash(202, fl.n_funcs(t, r, scheme))
    dev_rows = fl.to_device_rows(rows)
    ctx = fl.FastLSH(0)
    if args.bin_bits:
        ctx.configure(bin_bits=args.bin_bits)
    log(f"# generated {N} fingerprints in {gen_s:.1f}s; warmup {args.warmup}, steps {args.steps}")
    if args.autotune:
        ctx.configure(autotune=True)

    def step():
        return ctx.search(dev_rows, dim, t, r, scheme, a, b, L, v, occ_num, occ_den, graph=args.graph)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ctx.profile_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        out = step()
        log(f"# step {k + 1}/{args.steps}: {out[3].n_out} pairs")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = ctx.profile_read()
    work = ctx.last_work()
    calib_copy(args)
    ms_per_step = (t1 - t0) * 1000.0 / args.steps
    st = out[3]
    stage_ms, stage_launch = stage_table(prof, args.steps)
    dom = max(stage_ms, key=stage_ms.get)
    sig = sig_roofline(N, fl.n_funcs(t, r, scheme), scheme, stage_ms["signatures"], stage_launch["signatures"],
                       "k_sig<200,minmax>")
    if dom == "signatures":
        roof = dict(sig)
        traffic = kernel_traffic("k_sig_station90d", N)
        roof["traffic"] = traffic
        roof["traffic_unit"] = "bytes per launch (HBM, counter runs in profiles/)"
    else:
        roof = {"kernel": dom, "bound": "hbm", "achieved": None, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": None, "traffic": None, "launch_ms": round(stage_ms[dom], 3)}
    line = {
        "metric": "fingerprints/s through MinHash+LSH vote count",
        "value": round(N / (ms_per_step / 1000.0), 1),
        "unit": "fingerprints/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u32", "data": "synthetic",
        "config": {"workload": "one station, 90 days at 1 s lag: 7,776,000 fingerprints, 4096-dim, 200 bits, "
                               "Markov 70 %, 2,000 repeating sources; Min-Max t=100 r=4, lag 5, v=4, "
                               "occurrence filter 1 %",
                   "n": N, "tables": t, "rows": r, "scheme": "minmax", "min_lag": L, "min_votes": v,
                   "occ": f"{occ_num}/{occ_den}"},
        "candidate_pairs_per_s": round(st.e_raw / (ms_per_step / 1000.0), 1),
        "stats": stats_json(st),
        "stage_ms": {k: round(x, 3) for k, x in stage_ms.items()},
        "launch_shapes": ctx.config_used(),
        "roofline": roof,
        "k_pairs_tile": tile_roofline(work, st, stage_ms["big_pairs"], stage_launch["big_pairs"]),
    }
    line["cpu_baseline"] = cpu_baseline(lambda m: rows[:min(m, N)], dim, t, r, scheme, a, b, L, v, occ_num,
                                        occ_den, args, "the same workload")
    ctx.close()
    return line


def stats_json(st):
    """Search counters for the JSON line; n_distinct is null when the search
    was not asked to count distinct pairs (the library's all-ones marker)."""
    d = dict(st.__dict__)
    if d.get("n_distinct") == 2**64 - 1:
        d["n_distinct"] = None
    return d


def calib_copy(args):
    """A device-to-device copy of --calib-copy-mib MiB after the timed steps:
    the reference dispatch whose HBM counters calibrate FETCH_SIZE and
    WRITE_SIZE."""
    if not args.calib_copy_mib:
        return
    import torch
    src = torch.empty(args.calib_copy_mib << 20, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst


def upload_generated(spec, lo=0, hi=None, chunk=16_000_000):
    """Generate rows [lo, hi) of spec chunk by chunk into a pinned host buffer
    and copy each chunk into one device tensor (int16 [hi - lo, nnz])."""
    import numpy as np
    import torch

    import synth

    hi = spec.n if hi is None else hi
    dev = torch.empty((hi - lo, spec.nnz), dtype=torch.int16, device="cuda")
    pinned = torch.empty((min(chunk, hi - lo), spec.nnz), dtype=torch.int16, pin_memory=True)
    for c0 in range(lo, hi, chunk):
        c1 = min(hi, c0 + chunk)
        synth.generate(spec, c0, c1, out=pinned[: c1 - c0].numpy().view(np.uint16))
        dev[c0 - lo:c1 - lo].copy_(pinned[: c1 - c0])
        log(f"# generated rows {c0}..{c1}")
    del pinned
    return dev


def run_bounded(args):
    """One 5-year station with the bounded-memory search (tables in groups)."""
    import numpy as np
    import torch

    import synth
    import paper_1803_09835_amd as fl

    N = args.n or synth.STATION_5Y
    dim, t, r, scheme, L, v, occ_num, occ_den = 4096, 100, 4, fl.MINMAX, 5, 4, 1, 100
    spec = synth.long_station(n=N, seed=105)
    tg = time.time()
    dev = upload_generated(spec)
    log(f"# generated and uploaded {N} fingerprints in {time.time() - tg:.1f}s")
    a, b = fl.make_hash(205, fl.n_funcs(t, r, scheme))
    ctx = fl.FastLSH(0)
    if args.bin_bits:
        ctx.configure(bin_bits=args.bin_bits)
    gt = args.group_tables

    def step():
        return ctx.search_bounded(dev, dim, t, r, scheme, a, b, L, v, occ_num, occ_den, group_tables=gt)

    for k in range(args.warmup):
        out = step()
        log(f"# warm-up {k + 1}/{args.warmup}: {out[3].n_out} pairs")
    torch.cuda.synchronize()
    ctx.profile_enable(True)
    t0 = time.perf_counter()
    for k in range(args.steps):
        out = step()
        log(f"# step {k + 1}/{args.steps}: {out[3].n_out} pairs")
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1000.0 / args.steps
    prof = ctx.profile_read()
    work = ctx.last_work()
    calib_copy(args)
    stage_ms, stage_launch = stage_table(prof, args.steps)
    st = out[3]
    dom = max(stage_ms, key=stage_ms.get)
    sig = sig_roofline(N, fl.n_funcs(t, r, scheme), scheme, stage_ms["signatures"], stage_launch["signatures"],
                       "k_sig<200,minmax> (each table once)")
    tile = tile_roofline(work, st, stage_ms["big_pairs"], stage_launch["big_pairs"])
    tile["traffic"] = kernel_traffic("k_pairs_tile_station5y", N)
    tile["traffic_unit"] = "bytes per launch (HBM, counter runs in profiles/)"
    roof = tile if dom == "big_pairs" else (sig if dom == "signatures" else
                                             {"kernel": dom, "bound": "hbm", "achieved": None, "peak": HBM_PEAK_GBS,
                                              "unit": "GB/s", "frac": None, "traffic": None})
    line = {
        "metric": "fingerprints/s through MinHash+LSH vote count",
        "value": round(N / (ms / 1000.0), 1),
        "unit": "fingerprints/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u32", "data": "synthetic",
        "config": {"workload": "one station, 5 years at 1 s lag: 157,788,000 fingerprints, 4096-dim, 200 bits, "
                               "Markov 70 % in chains of 1 M, 20,000 repeating sources; Min-Max t=100 r=4, lag 5, "
                               f"v=4, occurrence filter 1 %; bounded-memory search, {gt} tables per group",
                   "n": N, "tables": t, "rows": r, "scheme": "minmax", "min_lag": L, "min_votes": v,
                   "occ": f"{occ_num}/{occ_den}", "group_tables": gt},
        "candidate_pairs_per_s": round(st.e_raw / (ms / 1000.0), 1),
        "stats": stats_json(st),
        "stage_ms": {k: round(x, 3) for k, x in stage_ms.items()},
        "dominant_stage": dom,
        "hbm_gb": {"fingerprints": round(dev.numel() * 2 / 1e9, 1),
                   "workspace": round(ctx.workspace_bytes() / 1e9, 1)},
        "roofline": roof,
        "k_sig": sig,
        "launch_shapes": ctx.config_used(),
    }
    if dom != "big_pairs":
        line["k_pairs_tile"] = tile
    ctx.close()
    del ctx
    line["cpu_baseline"] = cpu_baseline(lambda m: dev[:min(m, N)].cpu().numpy().view(np.uint16), dim, t, r,
                                        scheme, a, b, L, v, occ_num, occ_den, args, "the 5-year station")
    del dev
    return line


def serving_specs(S, n_hist, n_stream):
    import synth
    return [synth.Spec(n=n_hist + n_stream[s], seed=1040 + s, markov_keep=140, n_sources=4000, rep_min=3,
                       rep_max=40, jac_lo_milli=400, jac_hi_milli=900, chain_len=1_000_000) for s in range(S)]


def run_serving(args):
    """Stations of 180 days resident; 3,600-row chunks arrive as independent
    Poisson streams and are searched and inserted as they come."""
    import numpy as np
    import torch

    import synth
    import paper_1803_09835_amd as fl

    S, CH = args.stations, synth.CHUNK
    dim, t, r, scheme, L, v = 4096, 100, 4, fl.MINMAX, 5, 4
    n_hist = synth.STATION_180D if args.workload in ("headline",) or not args.n else args.n
    # arrivals: station s at rate/S per second (exponential gaps, seed 304)
    rng = np.random.default_rng(304)
    per = args.rate / S
    need = args.chunks // S + 40
    times = [np.cumsum(rng.exponential(1.0 / per, need)) for _ in range(S)]
    ev = sorted((times[s][c], s, c) for s in range(S) for c in range(need))[: args.chunks]
    ramp = 100  # further chunks per station, all offered at once
    used = [1 + max([c for _, s2, c in ev if s2 == s], default=-1) for s in range(S)]
    n_stream = [(u + ramp) * CH for u in used]
    a, b = fl.make_hash(204, fl.n_funcs(t, r, scheme))
    sv = fl.Server(dim, t, r, scheme, a, b, L, v, max_batch=8, max_chunk=CH, delta_rows=262144,
                   slack_rows=max(n_stream) + CH)
    streams = []
    tg = time.time()
    specs = serving_specs(S, n_hist, n_stream)
    for s, spec in enumerate(specs):
        hist = upload_generated(spec, 0, n_hist)
        sv.add_station(hist)
        del hist
        torch.cuda.empty_cache()
        rows = synth.generate(spec, n_hist, n_hist + n_stream[s])
        streams.append(fl.to_device_rows(rows))
        log(f"# station {s}: {n_hist} history rows resident, {n_stream[s]} stream rows ready "
            f"({time.time() - tg:.1f}s)")

    def run(events, label):
        """Submit (offset_s, station, chunk) at their times; latencies in ms."""
        t0 = sv.now_ns() + 50_000_000
        tickets = []
        last = time.perf_counter()
        for k, (off, s, c) in enumerate(events):
            at = t0 + int(off * 1e9)
            while True:
                now = sv.now_ns()
                if now >= at:
                    break
                if at - now > 2_000_000:
                    time.sleep((at - now - 1_000_000) / 1e9)
            tickets.append((at, sv.submit(s, streams[s][c * CH:(c + 1) * CH], at)))
            if time.perf_counter() - last > 10:
                last = time.perf_counter()
                log(f"# {label}: {k + 1}/{len(events)} submitted")
        lat, done, pairs = [], [], 0
        for at, tk in tickets:
            st, dn = sv.poll(tk, wait=True)
            sv.take(tk)
            lat.append((dn - at) / 1e6)
            done.append(dn)
            pairs += st.n_out
        span = (max(done) - min(at for at, _ in tickets)) / 1e9
        return np.array(lat), len(tickets) / span, pairs

    lat, thr, pairs = run([(off, s, c) for off, s, c in ev], f"offered {args.rate}/s")
    log(f"# offered load done: p50 {np.percentile(lat, 50):.2f} ms, p99 {np.percentile(lat, 99):.2f} ms")
    info1 = sv.info()
    sat_events = [(0.0, s, used[s] + c) for c in range(ramp) for s in range(S)]
    slat, sthr, _ = run(sat_events, "saturation")
    info2 = sv.info()
    batches = info2["batches"] - info1["batches"]
    line = {
        "metric": "fingerprints/s through MinHash+LSH vote count",
        "value": round(sthr * CH, 1),
        "unit": "fingerprints/s",
        "n_gpus": 1, "steps": len(sat_events), "warmup": 0,
        "ms_per_step": round(1000.0 / sthr, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u32", "data": "synthetic",
        "config": {"workload": f"serving: {S} stations of 180 days (15,552,000 fingerprints each, Markov 70 %, "
                               "4,000 repeating sources) resident; 3,600-fingerprint chunks searched against "
                               "everything before them and inserted; Min-Max t=100 r=4, lag 5, v=4, no occurrence "
                               "filter; value = fingerprints/s with all chunks offered at once (saturation)",
                   "stations": S, "history_rows": n_hist, "chunk_rows": CH, "tables": t, "rows": r,
                   "scheme": "minmax", "min_lag": L, "min_votes": v},
        "offered_load": {"chunks_per_s": args.rate, "chunks": len(ev), "sustained_chunks_per_s": round(thr, 2),
                         "latency_ms": {"p50": round(float(np.percentile(lat, 50)), 3),
                                        "p99": round(float(np.percentile(lat, 99)), 3),
                                        "mean": round(float(lat.mean()), 3), "max": round(float(lat.max()), 3)},
                         "pairs": int(pairs)},
        "saturation": {"chunks": len(sat_events), "chunks_per_s": round(sthr, 2), "batches": batches,
                       "mean_batch": round(len(sat_events) / max(batches, 1), 2),
                       "fingerprints_per_s": round(sthr * CH, 1),
                       "latency_ms": {"p50": round(float(np.percentile(slat, 50)), 3),
                                      "p99": round(float(np.percentile(slat, 99)), 3)}},
        "hbm_gb": {"resident": round(info2["resident_bytes"] / 1e9, 1),
                   "workspace": round(info2["workspace_bytes"] / 1e9, 2),
                   "stream_rows": round(sum(x.numel() * 2 for x in streams) / 1e9, 1)},
        "roofline": None,
    }
    sv.close()
    del sv, streams
    return line, specs[0]


def run_plain_chunk(spec, reps=3):
    """The plain path for one chunk: a full search of a served station's
    history plus its first chunk (15,555,600 fingerprints of that station's
    rows), whose pairs with the later member in the chunk are that chunk's
    result.  Returns its time."""
    import torch

    import synth
    import paper_1803_09835_amd as fl

    CH = synth.CHUNK
    n_hist = synth.STATION_180D
    dim, t, r, scheme, L, v = 4096, 100, 4, fl.MINMAX, 5, 4
    dev = upload_generated(spec, 0, n_hist + CH)
    a, b = fl.make_hash(204, fl.n_funcs(t, r, scheme))
    ctx = fl.FastLSH(0)
    ctx.search(dev, dim, t, r, scheme, a, b, L, v)
    torch.cuda.synchronize()
    ms = []
    for _ in range(reps):
        t0 = time.perf_counter()
        out = ctx.search(dev, dim, t, r, scheme, a, b, L, v)
        torch.cuda.synchronize()
        ms.append((time.perf_counter() - t0) * 1000.0)
    n_chunk = int((out[1] >= n_hist).sum().item())
    log(f"# plain search of history + chunk: {min(ms):.1f} ms, {n_chunk} pairs end in the chunk")
    ctx.close()
    del dev, ctx
    return {"n": n_hist + CH, "ms": round(sorted(ms)[len(ms) // 2], 3), "reps": reps,
            "pairs_ending_in_chunk": n_chunk}


def run_batched(args):
    """12 stations of the uniform generator (50 events x 5 copies each), one
    batched search against 12 sequential single-station searches."""
    import torch

    import synth
    import paper_1803_09835_amd as fl

    dim, t, r, scheme, L, v = 4096, 20, 4, fl.MINHASH, 5, 2
    sizes = [m * 1_000_000 for m in synth.BATCH_LENGTHS_M]
    specs = [synth.tiny_uniform(n=n, seed=1030 + s) for s, n in enumerate(sizes)]
    # one station after another (each generation is OpenMP-parallel inside),
    # before the GPU is touched
    tg = time.time()
    host = []
    for s, sp in enumerate(specs):
        host.append(synth.generate(sp))
        log(f"# station {s}: {sp.n} rows generated ({time.time() - tg:.1f}s)")
    dev = [fl.to_device_rows(h) for h in host]
    N = sum(sizes)
    log(f"# generated and uploaded {N} fingerprints in {time.time() - tg:.1f}s")
    a, b = fl.make_hash(201, fl.n_funcs(t, r, scheme))
    ctx_b = fl.FastLSH(0)
    ctx_s = fl.FastLSH(0)
    if args.bin_bits:
        ctx_b.configure(bin_bits=args.bin_bits)
        ctx_s.configure(bin_bits=args.bin_bits)
    if args.autotune:
        ctx_b.configure(autotune=True)
        ctx_s.configure(autotune=True)

    def batched():
        return ctx_b.search_batched(dev, dim, t, r, scheme, a, b, L, v, graph=args.graph)

    def sequential():
        return [ctx_s.search(d, dim, t, r, scheme, a, b, L, v, graph=args.graph) for d in dev]

    def timed(fn, name, ctx):
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        ctx.profile_enable(True)
        t0 = time.perf_counter()
        for k in range(args.steps):
            out = fn()
            log(f"# {name} step {k + 1}/{args.steps}")
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1000.0 / args.steps
        prof = ctx.profile_read()
        return out, ms, {k: round(x / args.steps, 3) for k, (x, n) in prof.items()}, prof

    out_b, ms_b, stage_b, prof_b = timed(batched, "batched", ctx_b)
    out_s, ms_s, stage_s, _ = timed(sequential, "sequential", ctx_s)
    # the two must agree pair for pair
    offs = out_b[3]
    same = all(torch.equal(out_b[q][offs[s]:offs[s + 1]], out_s[s][q]) for s in range(len(dev)) for q in range(3))
    same = same and all(out_b[4][s] == out_s[s][3] for s in range(len(dev)))

    dom = max(stage_b, key=stage_b.get)
    if prof_b["signatures"][1]:
        roof = sig_roofline(N, fl.n_funcs(t, r, scheme), scheme, prof_b["signatures"][0] / args.steps,
                            prof_b["signatures"][1] / args.steps, "k_sig<200,minhash> (all stations)")
        roof["traffic"] = None
    else:  # kernels inside the replayed graph are not timed one by one
        roof = None
    line = {
        "metric": "fingerprints/s through MinHash+LSH vote count",
        "value": round(N / (ms_b / 1000.0), 1),
        "unit": "fingerprints/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_b, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u32", "data": "synthetic",
        "config": {"workload": "12 stations of 1-8, 10, 12, 14, 16 M fingerprints (88 M), uniform 200-of-4096 "
                               "background with 50 events x 5 copies keeping 160 bits each; MinHash t=20 r=4, "
                               "lag 5, v=2, no occurrence filter; one batched search",
                   "n": N, "stations": len(sizes), "tables": t, "rows": r, "scheme": "minhash", "min_lag": L,
                   "min_votes": v, "graph": args.graph, "autotune": args.autotune},
        "sequential_ms_per_step": round(ms_s, 3),
        "speedup_vs_sequential": round(ms_s / ms_b, 3),
        "identical_to_sequential": bool(same),
        "n_out": int(offs[-1]),
        "e_raw": int(sum(st.e_raw for st in out_b[4])),
        "stage_ms": stage_b,
        "sequential_stage_ms": stage_s,
        "launch_shapes": ctx_b.config_used(),
        "dominant_stage": dom,
        "roofline": roof,
    }
    line["cpu_baseline"] = cpu_baseline(lambda m: host[0][:min(m, len(host[0]))], dim, t, r, scheme, a, b, L, v,
                                        0, 0, args, "the 1 M-fingerprint station")
    ctx_b.close()
    ctx_s.close()
    return line


def run_alignment(args):
    """Three channels of one 90-day station (shared repeating sources,
    per-channel background), each searched with a lenient threshold (v = 2);
    one step = the channel merge of the three outputs (combined similarity
    at least 6) plus the station clusters of the merged entries."""
    import numpy as np
    import torch

    import synth
    import paper_1803_09835_amd as fl

    N = args.n or synth.STATION_90D
    dim, t, r, scheme, L, v = 4096, 100, 4, fl.MINMAX, 5, 2
    min_sim, gap, width, min_entries = 6, 10, 3, 2
    a, b = fl.make_hash(202, fl.n_funcs(t, r, scheme))
    ctx = fl.FastLSH(0)
    if args.bin_bits:
        ctx.configure(bin_bits=args.bin_bits)
    chans = []
    for ch in range(3):
        spec = synth.Spec(n=N, seed=102, markov_keep=140, n_sources=max(1, round(2000 * N / synth.STATION_90D)),
                          rep_min=3, rep_max=40, jac_lo_milli=400, jac_hi_milli=900, channel=ch)
        dev = fl.to_device_rows(synth.generate(spec))
        oi, oj, ov, st = ctx.search(dev, dim, t, r, scheme, a, b, L, v, 1, 100)
        chans.append((oi.clone(), oj.clone(), ov.clone()))
        del dev, oi, oj, ov
        log(f"# channel {ch}: {st.n_out} pairs at v >= {v}")
    torch.cuda.empty_cache()
    total = sum(c[0].numel() for c in chans)

    def step():
        dt, x, sm = ctx.channel_merge(chans, N, min_sim)
        cl = ctx.station_clusters(dt, x, sm, gap, width, min_entries, 0)
        return dt, x, sm, cl

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ctx.profile_enable(True)
    t0 = time.perf_counter()
    for k in range(args.steps):
        out = step()
        log(f"# step {k + 1}/{args.steps}: {out[0].numel()} merged entries, {out[3].shape[0]} clusters")
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1000.0 / args.steps
    prof = ctx.profile_read()
    stage_ms, _ = stage_table(prof, args.steps)
    merged, n_cl = out[0].numel(), out[3].shape[0]
    # algorithmic bytes of the merge: the 9-byte pairs read, one LSD sort of
    # 12-byte records (8-byte key, 4-byte sim: read and written once per
    # 8-bit digit of the two ids, plus a 8-byte key read per histogram), the
    # merged 12-byte entries written
    nb = max(1, (N - 1).bit_length())
    passes = 2 * ((nb + 7) // 8)
    algo = total * 9 + total * passes * (24 + 8) + merged * 12
    mgbs = algo / (stage_ms["channel_merge"] / 1000.0) / 1e9
    line = {
        "metric": "fingerprint pairs/s through the channel merge and station clustering",
        "value": round(total / (ms / 1000.0), 1),
        "unit": "pairs/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u32", "data": "synthetic",
        "config": {"workload": "three channels of one station, 90 days at 1 s lag (7,776,000 fingerprints each, "
                               "shared repeating sources, per-channel Markov background); each searched with "
                               "Min-Max t=100 r=4, lag 5, v=2, filter 1 %; channel merge at combined similarity "
                               f">= {min_sim}, clusters with gap {gap}, width {width}, at least {min_entries} entries",
                   "n": N, "channels": 3, "pairs_in": total, "min_sim": min_sim, "max_gap": gap,
                   "max_width": width, "min_entries": min_entries},
        "merged_entries": merged, "clusters": n_cl,
        "stage_ms": {k: round(x, 3) for k, x in stage_ms.items() if x},
        "roofline": {"kernel": "channel merge (pack, radix passes, run sums, compaction)", "bound": "hbm",
                     "achieved": round(mgbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(mgbs / HBM_PEAK_GBS, 4), "traffic": None, "algorithmic_bytes": algo,
                     "radix_passes": passes},
    }
    import oracle
    host = [(c[0].cpu().numpy().view(np.uint32), c[1].cpu().numpy().view(np.uint32), c[2].cpu().numpy())
            for c in chans]
    tc = time.perf_counter()
    wdt, wx, ws = oracle.channel_merge(host, min_sim)
    oracle.station_clusters(wdt, wx, ws, gap, width, min_entries, 0)
    cpu_s = time.perf_counter() - tc
    line["cpu_baseline"] = {"value": round(total / cpu_s, 1), "unit": "pairs/s", "cores": 1, "kind": "oracle",
                            "cpu": cpu_model(),
                            "sample": f"the whole input ({total} pairs), merge and clusters in {cpu_s:.1f} s "
                                      "(single-threaded code)"}
    ctx.close()
    return line


def run_query(args, nq=1000):
    """Query-only hashing: nq queries (half of them rows of the station,
    half independent fingerprints) against the 90-day station; one step =
    one query-only search.  The plain search of station plus queries (tables
    over everything) is timed beside it."""
    import numpy as np
    import torch

    import synth
    import paper_1803_09835_amd as fl

    N = args.n or synth.STATION_90D
    dim, t, r, scheme, v = 4096, 100, 4, fl.MINMAX, 4
    rows = synth.generate(synth.station(n=N, seed=102))
    rng = np.random.default_rng(306)
    qrows = np.concatenate([rows[rng.choice(N, nq // 2, replace=False)],
                            synth.generate(synth.Spec(n=nq - nq // 2, seed=307))])
    a, b = fl.make_hash(202, fl.n_funcs(t, r, scheme))
    d, q = fl.to_device_rows(rows), fl.to_device_rows(qrows)
    ctx = fl.FastLSH(0)

    def step():
        return ctx.query(q, d, dim, t, r, scheme, a, b, v)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ctx.profile_enable(True)
    t0 = time.perf_counter()
    for k in range(args.steps):
        out = step()
        log(f"# step {k + 1}/{args.steps}: {out[3].n_out} pairs, {out[3].e_raw} matches")
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1000.0 / args.steps
    prof = ctx.profile_read()
    stage_ms, stage_launch = stage_table(prof, args.steps)
    both = torch.cat([d, q])
    ctx.search(both, dim, t, r, scheme, a, b, 1, v)
    torch.cuda.synchronize()
    tp = time.perf_counter()
    ctx.search(both, dim, t, r, scheme, a, b, 1, v)
    torch.cuda.synchronize()
    plain_ms = (time.perf_counter() - tp) * 1000.0
    sig = sig_roofline(N, fl.n_funcs(t, r, scheme), scheme, stage_ms["signatures"], stage_launch["signatures"],
                       "k_sig<200,minmax> (dataset and queries)")
    line = {
        "metric": "dataset fingerprints/s through query-only hashing",
        "value": round(N / (ms / 1000.0), 1),
        "unit": "fingerprints/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u32", "data": "synthetic",
        "config": {"workload": f"{nq} queries (half of them rows of the station, half independent) against one "
                               "station, 90 days at 1 s lag (7,776,000 fingerprints); Min-Max t=100 r=4, v=4; only "
                               "the queries hashed into tables",
                   "n": N, "queries": nq, "tables": t, "rows": r, "min_votes": v},
        "pairs": out[3].n_out, "matches": out[3].e_raw,
        "stage_ms": {k: round(x, 3) for k, x in stage_ms.items() if x},
        "plain_search_of_dataset_and_queries_ms": round(plain_ms, 3),
        "speedup_vs_plain_search": round(plain_ms / ms, 2),
        "roofline": sig,
    }
    import oracle
    ns = min(200_000, N)
    tc = time.perf_counter()
    oracle.query(qrows, rows[:ns], dim, t, r, oracle.MINMAX, a, b, v)
    cpu_s = time.perf_counter() - tc
    line["cpu_baseline"] = {"value": round(ns / cpu_s, 1), "unit": "fingerprints/s", "cores": oracle.max_threads(),
                            "kind": "oracle", "cpu": cpu_model(),
                            "sample": f"the {nq} queries against the first {ns} fingerprints, {cpu_s:.1f} s"}
    ctx.close()
    return line


def run_partitioned(args, parts=3):
    """The 90-day station searched in three partitions (months) with the
    dynamic occurrence filter at 1 % of each partition; one step = one
    partitioned search.  The plain search (static filter) is timed beside it."""
    import torch

    import synth
    import paper_1803_09835_amd as fl

    N = args.n or synth.STATION_90D
    dim, t, r, scheme, L, v = 4096, 100, 4, fl.MINMAX, 5, 4
    rows = synth.generate(synth.station(n=N, seed=102))
    a, b = fl.make_hash(202, fl.n_funcs(t, r, scheme))
    d = fl.to_device_rows(rows)
    ctx = fl.FastLSH(0)

    def step():
        return ctx.search_partitioned(d, dim, t, r, scheme, a, b, L, v, 1, 100, n_partitions=parts)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ctx.profile_enable(True)
    t0 = time.perf_counter()
    for k in range(args.steps):
        out = step()
        log(f"# step {k + 1}/{args.steps}: {out[3].n_out} pairs, {out[3].n_flagged} excluded")
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1000.0 / args.steps
    prof = ctx.profile_read()
    stage_ms, _ = stage_table(prof, args.steps)
    ctx.search(d, dim, t, r, scheme, a, b, L, v, 1, 100)
    torch.cuda.synchronize()
    tp = time.perf_counter()
    plain = ctx.search(d, dim, t, r, scheme, a, b, L, v, 1, 100)
    torch.cuda.synchronize()
    plain_ms = (time.perf_counter() - tp) * 1000.0
    line = {
        "metric": "fingerprints/s through the partitioned search with the dynamic occurrence filter",
        "value": round(N / (ms / 1000.0), 1),
        "unit": "fingerprints/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u32", "data": "synthetic",
        "config": {"workload": "one station, 90 days at 1 s lag (7,776,000 fingerprints) in three partitions of 30 "
                               "days; Min-Max t=100 r=4, lag 5, v=4; dynamic occurrence filter at 1 % of each "
                               "partition", "n": N, "partitions": parts, "tables": t, "min_votes": v},
        "stats": stats_json(out[3]),
        "same_pairs_as_plain_search": bool(all(torch.equal(x, y) for x, y in zip(out[:3], plain[:3]))),
        "stage_ms": {k: round(x, 3) for k, x in stage_ms.items() if x},
        "plain_search_ms": round(plain_ms, 3),
        "roofline": None,
    }
    ctx.close()
    return line


def run_fingerprints(args):
    """Fingerprint extraction of one channel, 90 days at 100 Hz (777,600,000
    samples: Gaussian noise with 2,000 repeating sources of 3-40 events),
    window 200, hop 10, band bins 4-35, 128 frames per fingerprint averaged
    in pairs, 1 s lag, K = 200: 7,776,000 fingerprints of 4,096 bits.  The
    normalization statistics use a seeded 1 % sample of the fingerprints.
    One step = one extraction from samples in HBM to fingerprints in HBM."""
    import numpy as np
    import torch

    import synth
    import paper_1803_09835_amd as fl

    spec = synth.station_waveform(days=(args.n / 86_400 / 100) if args.n else 90)
    window, hop, rows, fp_frames, fp_lag, top_k = 200, 10, 32, 128, 10, 200
    n = spec.n
    dev = torch.empty(n, dtype=torch.float32, device="cuda")
    pinned = torch.empty(min(n, 100_000_000), dtype=torch.float32, pin_memory=True)
    tg = time.time()
    for lo in range(0, n, pinned.numel()):
        hi = min(n, lo + pinned.numel())
        synth.waveform(spec, lo, hi, out=pinned[: hi - lo].numpy())
        dev[lo:hi].copy_(pinned[: hi - lo])
    del pinned
    frames = (n - window) // hop + 1
    nf = (frames - fp_frames) // fp_lag + 1
    rng = np.random.default_rng(405)
    sample = np.sort(rng.choice(nf, max(1, nf // 100), replace=False))
    log(f"# waveform of {n} samples in {time.time() - tg:.1f}s; {nf} fingerprints, sample {len(sample)}")
    ctx = fl.FastLSH(0)

    def step():
        return ctx.fingerprints(dev, sample)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ctx.profile_enable(True)
    t0 = time.perf_counter()
    for k in range(args.steps):
        out, cnt = step()
        log(f"# step {k + 1}/{args.steps}: {out.shape[0]} fingerprints")
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1000.0 / args.steps
    prof = ctx.profile_read()
    stage_ms, _ = stage_table(prof, args.steps)
    flop = frames * rows * 2 * window * 2  # cosine and sine rows of every kept bin: one FMA per sample each
    tf = flop / (stage_ms["spectrogram"] / 1000.0) / 1e12
    full = int((cnt == top_k).sum().item())
    line = {
        "metric": "fingerprints/s through fingerprint extraction",
        "value": round(nf / (ms / 1000.0), 1),
        "unit": "fingerprints/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "one channel, 90 days at 100 Hz (777,600,000 samples, Gaussian noise, 2,000 repeating "
                               "sources of 3-40 P/S events); STFT window 200 hop 10, bins 4-35, 128 frames averaged "
                               "in pairs, 1 s lag, 2-D Haar, MAD over a 1 % sample, K = 200",
                   "samples": n, "fingerprints": nf, "sample": len(sample), "dim": 2 * rows * fp_frames // 2,
                   "top_k": top_k},
        "fingerprints_with_k_bits": full,
        "stage_ms": {k: round(x, 3) for k, x in stage_ms.items() if x},
        "roofline": {"kernel": "k_stft_mfma (with its basis rows)", "bound": "mfma", "achieved": round(tf, 2),
                     "peak": 157.3, "unit": "TFLOP/s (fp32 MFMA)", "frac": round(tf / 157.3, 4), "traffic": None,
                     "flop_per_frame": rows * 4 * window, "frames": frames},
    }
    from oracle import fingerprint as ofp
    p = ofp.FpParams()
    sl = 100 * 3600  # one hour of samples
    xs = dev[:sl].cpu().numpy()
    nfs = ofp.n_fingerprints(sl, p)
    tc = time.perf_counter()
    ofp.fingerprints(xs.astype(np.float64), p, np.arange(0, nfs, 100), np.arange(nfs))
    cpu_s = time.perf_counter() - tc
    line["cpu_baseline"] = {"value": round(nfs / cpu_s, 1), "unit": "fingerprints/s", "cores": 1, "kind": "oracle",
                            "cpu": cpu_model(),
                            "sample": f"the first hour ({nfs} fingerprints, statistics of every 100th), {cpu_s:.1f} s "
                                      "in float64 numpy (one thread)"}
    ctx.close()
    return line


if __name__ == "__main__":
    main()
