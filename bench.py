#!/usr/bin/env python3
"""Throughput of the LSH similarity search on one MI355X.

Workload: one station, 90 days of fingerprints at a 1 s lag (7,776,000
fingerprints, 4096-dim, 200 set bits each; Markov background keeping 70 % of
the previous fingerprint; 2,000 repeating sources with 3-40 copies whose
Jaccard similarity to the template is U[0.4, 0.9]).  Min-Max hash, t = 100
tables, r = 4 rows (2 functions per table), self-match lag 5, at least 4
votes, occurrence filter at 1 % of N.

One step = one full search: signatures, grouping of all 100 tables, bucket
segmentation and occurrence filter, in-bucket pair votes, threshold and
canonical sort, from fingerprints resident in HBM to the sorted pairs in HBM
and the pair count on the host.  value = fingerprints / second.

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

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


def sig_traffic(n):
    """HBM bytes per signature launch from the committed counter figures, or
    None when they were taken for another size or on different kernel code."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "k_sig_station90d_traffic.txt")
    if not os.path.exists(path):
        return None
    kv = dict(l.strip().split("=", 1) for l in open(path) if "=" in l and not l.startswith("#"))
    src = b"".join(open(os.path.join(ROOT, "paper_1803_09835_amd", "csrc", f), "rb").read()
                   for f in ("sig.hip", "common.hpp"))
    if int(kv.get("n", -1)) != n or kv.get("source_sha256") != hashlib.sha256(src).hexdigest():
        return None
    return int(kv["fetch_bytes"]) + int(kv["write_bytes"])


def parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--chunks", type=int, default=3000, help="serving workload: chunks at the offered load")
    ap.add_argument("--rate", type=float, default=40.0, help="serving workload: offered chunks/s (all stations)")
    ap.add_argument("--stations", type=int, default=8, help="serving workload: stations")
    ap.add_argument("--workload", choices=("station", "batched", "bounded", "serving"), default="station",
                    help="station: one 90-day station (default); batched: 12 stations of 1-16 M fingerprints "
                         "in one search, against 12 sequential searches; bounded: one 5-year station "
                         "(157,788,000 fingerprints) with tables taken 10 at a time; serving: 8 stations of "
                         "180 days resident, 3,600-row chunks arriving as Poisson streams")
    ap.add_argument("--group-tables", type=int, default=10, help="bounded workload: tables per group")
    ap.add_argument("--graph", action="store_true", help="replay the captured graph of the search prefix")
    ap.add_argument("--autotune", action="store_true", help="tune launch shapes on the first (warm-up) search")
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=7_776_000, help="fingerprints (default: 90 days at 1 s)")
    ap.add_argument("--cpu-sample", type=int, default=1_000_000,
                    help="fingerprints of the same workload the CPU oracle is timed on (0: skip)")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="after timing, copy this many MiB device-to-device with a plain copy kernel "
                         "(reference dispatch for HBM counter calibration)")
    return ap.parse_args()


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "fast_lsh searches on one GPU; sharding a search over several GPUs is not "
                                   "implemented", "n_gpus": args.gpus}))
        sys.exit(2)
    if args.workload == "bounded":
        return main_bounded(args)
    if args.workload == "serving":
        return main_serving(args)
    if args.workload == "batched":
        # This mode's process ended with a host segmentation fault within its
        # first seconds (while generating the 12 stations from 12 host threads),
        # once in three runs; the cause is not known, so it stays switched off.
        print(json.dumps({"error": "the batched workload mode is switched off: its process crashed on the host "
                                   "during data generation and the cause is not yet known",
                          "workload": "batched"}))
        sys.exit(2)

    import numpy as np
    import torch

    import synth
    import paper_1803_09835_amd as fl

    N = args.n
    dim, t, r, scheme = 4096, 100, 4, fl.MINMAX
    L, v, occ_num, occ_den = 5, 4, 1, 100
    spec = synth.station(n=N, seed=102)
    tg = time.time()
    rows = synth.generate(spec)
    gen_s = time.time() - tg
    a, b = fl.make_hash(202, fl.n_funcs(t, r, scheme))
    dev_rows = fl.to_device_rows(rows)
    ctx = fl.FastLSH(0)
    print(f"# generated {N} fingerprints in {gen_s:.1f}s; warmup {args.warmup}, steps {args.steps}",
          file=sys.stderr, flush=True)

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
        print(f"# step {k + 1}/{args.steps}: {out[3].n_out} pairs", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = ctx.profile_read()
    if args.calib_copy_mib:
        src = torch.empty(args.calib_copy_mib << 20, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    ms_per_step = (t1 - t0) * 1000.0 / args.steps
    st = out[3]
    value = N / (ms_per_step / 1000.0)

    # Dominant kernel and its roofline (kernel time from HIP events on the
    # context stream over the timed steps).
    stage_ms = {k: ms / args.steps for k, (ms, n) in prof.items()}
    stage_launch = {k: n / args.steps for k, (ms, n) in prof.items()}
    dom = max(stage_ms, key=stage_ms.get)
    if dom == "signatures" and stage_launch[dom]:
        evals = N * fl.n_funcs(t, r, scheme) * 200  # (fingerprint, function, set element)
        per_launch_ms = stage_ms[dom] / max(stage_launch[dom], 1)
        achieved = evals * OPS_PER_EVAL[scheme] / (per_launch_ms / 1000.0) / 1e12
        traffic = sig_traffic(N)
        roof = {"kernel": "k_sig<200,minmax>", "bound": "alu", "achieved": round(achieved, 2),
                "peak": round(INT_PEAK_TOPS, 2), "unit": "TOP/s (int32)",
                "frac": round(achieved / INT_PEAK_TOPS, 4), "traffic": traffic,
                "traffic_unit": "bytes per launch (HBM, counter runs in profiles/)",
                "traffic_gbs": round(traffic / (per_launch_ms / 1000.0) / 1e9, 1) if traffic else None,
                "evals_per_s": evals / (per_launch_ms / 1000.0), "launch_ms": round(per_launch_ms, 3)}
    else:
        roof = {"kernel": dom, "bound": "hbm", "achieved": None, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": None, "traffic": None, "launch_ms": round(stage_ms[dom], 3)}

    line = {
        "metric": "fingerprints/s through MinHash+LSH vote count",
        "value": round(value, 1),
        "unit": "fingerprints/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": "one station, 90 days at 1 s lag: 7,776,000 fingerprints, 4096-dim, 200 bits, "
                               "Markov 70 %, 2,000 repeating sources; Min-Max t=100 r=4, lag 5, v=4, "
                               "occurrence filter 1 %",
                   "n": N, "tables": t, "rows": r, "scheme": "minmax", "min_lag": L, "min_votes": v,
                   "occ": f"{occ_num}/{occ_den}"},
        "candidate_pairs_per_s": round(st.e_raw / (ms_per_step / 1000.0), 1),
        "stats": st.__dict__,
        "stage_ms": {k: round(x, 3) for k, x in stage_ms.items()},
        "launch_shapes": ctx.config_used(),
        "roofline": roof,
    }

    if args.cpu_sample > 0:
        import oracle
        ns = min(args.cpu_sample, N)
        sample = rows[:ns]
        tc = time.perf_counter()
        _, _, _, ost = oracle.search(sample, dim, t, r, oracle.MINMAX, a, b, L, v, occ_num, occ_den)
        cpu_s = time.perf_counter() - tc
        line["cpu_baseline"] = {
            "value": round(ns / cpu_s, 1), "unit": "fingerprints/s", "cores": oracle.max_threads(),
            "kind": "oracle",
            "sample": f"first {ns} fingerprints of the same workload, full search (signatures + votes), "
                      f"{cpu_s:.1f} s; the pair work grows with N so a slice under-states the full-size cost",
        }
    print(json.dumps(line), flush=True)


def main_batched(args):
    """12 stations of the uniform generator (50 events x 5 copies each), one
    batched search against 12 sequential single-station searches."""
    from concurrent.futures import ThreadPoolExecutor

    import numpy as np
    import torch

    import synth
    import paper_1803_09835_amd as fl

    dim, t, r, scheme, L, v = 4096, 20, 4, fl.MINHASH, 5, 2
    sizes = [m * 1_000_000 for m in synth.BATCH_LENGTHS_M]
    specs = [synth.tiny_uniform(n=n, seed=1030 + s) for s, n in enumerate(sizes)]
    tg = time.time()
    with ThreadPoolExecutor(max_workers=12) as ex:
        host = list(ex.map(synth.generate, specs))
    dev = []
    for h in host:
        dev.append(fl.to_device_rows(h))
    N = sum(sizes)
    print(f"# generated and uploaded {N} fingerprints in {time.time() - tg:.1f}s", file=sys.stderr, flush=True)
    a, b = fl.make_hash(201, fl.n_funcs(t, r, scheme))
    ctx_b = fl.FastLSH(0)
    ctx_s = fl.FastLSH(0)
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
            print(f"# {name} step {k + 1}/{args.steps}", file=sys.stderr, flush=True)
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

    evals = N * fl.n_funcs(t, r, scheme) * 200
    dom = max(stage_b, key=stage_b.get)
    if prof_b["signatures"][1]:
        sig_launch_ms = prof_b["signatures"][0] / prof_b["signatures"][1]
        achieved = evals * OPS_PER_EVAL[scheme] / (sig_launch_ms / 1000.0) / 1e12
        roof = {"kernel": "k_sig<200,minhash> (all stations)", "bound": "alu", "achieved": round(achieved, 2),
                "peak": round(INT_PEAK_TOPS, 2), "unit": "TOP/s (int32)",
                "frac": round(achieved / INT_PEAK_TOPS, 4), "traffic": None, "launch_ms": round(sig_launch_ms, 3)}
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
    if args.cpu_sample > 0:
        import oracle
        rows = host[0][: min(args.cpu_sample, len(host[0]))]
        tc = time.perf_counter()
        oracle.search(rows, dim, t, r, oracle.MINHASH, a, b, L, v)
        cpu_s = time.perf_counter() - tc
        line["cpu_baseline"] = {"value": round(len(rows) / cpu_s, 1), "unit": "fingerprints/s",
                                "cores": oracle.max_threads(), "kind": "oracle",
                                "sample": f"the 1 M-fingerprint station searched alone, {cpu_s:.1f} s"}
    print(json.dumps(line), flush=True)


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
        print(f"# generated rows {c0}..{c1}", file=sys.stderr, flush=True)
    del pinned
    return dev


def main_bounded(args):
    """One 5-year station with the bounded-memory search (tables in groups)."""
    import numpy as np
    import torch

    import synth
    import paper_1803_09835_amd as fl

    N = synth.STATION_5Y if args.n == 7_776_000 else args.n
    dim, t, r, scheme, L, v, occ_num, occ_den = 4096, 100, 4, fl.MINMAX, 5, 4, 1, 100
    spec = synth.long_station(n=N, seed=105)
    tg = time.time()
    dev = upload_generated(spec)
    print(f"# generated and uploaded {N} fingerprints in {time.time() - tg:.1f}s", file=sys.stderr, flush=True)
    a, b = fl.make_hash(205, fl.n_funcs(t, r, scheme))
    ctx = fl.FastLSH(0)
    gt = args.group_tables

    def step():
        return ctx.search_bounded(dev, dim, t, r, scheme, a, b, L, v, occ_num, occ_den, group_tables=gt)

    for k in range(args.warmup):
        out = step()
        print(f"# warm-up {k + 1}/{args.warmup}: {out[3].n_out} pairs", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    ctx.profile_enable(True)
    t0 = time.perf_counter()
    for k in range(args.steps):
        out = step()
        print(f"# step {k + 1}/{args.steps}: {out[3].n_out} pairs", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1000.0 / args.steps
    prof = ctx.profile_read()
    stage_ms = {k: round(x / args.steps, 3) for k, (x, n) in prof.items()}
    st = out[3]
    # signature kernel: 2 x t tables of work per search (both passes)
    sig_ms = prof["signatures"][0] / args.steps
    evals = 2 * N * fl.n_funcs(t, r, scheme) * 200
    sig_tops = evals * OPS_PER_EVAL[scheme] / (sig_ms / 1000.0) / 1e12
    dom = max(stage_ms, key=stage_ms.get)
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
        "stats": st.__dict__,
        "stage_ms": stage_ms,
        "dominant_stage": dom,
        "hbm_gb": {"fingerprints": round(dev.numel() * 2 / 1e9, 1),
                   "workspace": round(ctx.workspace_bytes() / 1e9, 1)},
        "roofline": {"kernel": "k_sig<200,minmax> (both passes)", "bound": "alu", "achieved": round(sig_tops, 2),
                     "peak": round(INT_PEAK_TOPS, 2), "unit": "TOP/s (int32)",
                     "frac": round(sig_tops / INT_PEAK_TOPS, 4), "traffic": None,
                     "launch_ms": round(sig_ms / max(prof["signatures"][1] / args.steps, 1), 3)},
    }
    if args.cpu_sample > 0:
        import oracle
        ns = min(args.cpu_sample, N)
        rows = dev[:ns].cpu().numpy().view(np.uint16)
        tc = time.perf_counter()
        oracle.search(rows, dim, t, r, oracle.MINMAX, a, b, L, v, occ_num, occ_den)
        cpu_s = time.perf_counter() - tc
        line["cpu_baseline"] = {"value": round(ns / cpu_s, 1), "unit": "fingerprints/s",
                                "cores": oracle.max_threads(), "kind": "oracle",
                                "sample": f"first {ns} fingerprints searched alone, {cpu_s:.1f} s; the pair work "
                                          f"grows with N, so a slice over-states the CPU rate at full size"}
    print(json.dumps(line), flush=True)


def main_serving(args):
    """Stations of 180 days resident; 3,600-row chunks arrive as independent
    Poisson streams and are searched and inserted as they come."""
    import numpy as np
    import torch

    import synth
    import paper_1803_09835_amd as fl

    S, CH = args.stations, synth.CHUNK
    dim, t, r, scheme, L, v = 4096, 100, 4, fl.MINMAX, 5, 4
    n_hist = synth.STATION_180D if args.n == 7_776_000 else args.n
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
    for s in range(S):
        spec = synth.Spec(n=n_hist + n_stream[s], seed=1040 + s, markov_keep=140, n_sources=4000, rep_min=3,
                          rep_max=40, jac_lo_milli=400, jac_hi_milli=900, chain_len=1_000_000)
        hist = upload_generated(spec, 0, n_hist)
        sv.add_station(hist)
        del hist
        torch.cuda.empty_cache()
        rows = synth.generate(spec, n_hist, n_hist + n_stream[s])
        streams.append(fl.to_device_rows(rows))
        print(f"# station {s}: {n_hist} history rows resident, {n_stream[s]} stream rows ready "
              f"({time.time() - tg:.1f}s)", file=sys.stderr, flush=True)
    info0 = sv.info()

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
                print(f"# {label}: {k + 1}/{len(events)} submitted", file=sys.stderr, flush=True)
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
    print(f"# offered load done: p50 {np.percentile(lat, 50):.2f} ms, p99 {np.percentile(lat, 99):.2f} ms",
          file=sys.stderr, flush=True)
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
                       "latency_ms": {"p50": round(float(np.percentile(slat, 50)), 3),
                                      "p99": round(float(np.percentile(slat, 99)), 3)}},
        "hbm_gb": {"resident": round(info2["resident_bytes"] / 1e9, 1),
                   "workspace": round(info2["workspace_bytes"] / 1e9, 2),
                   "stream_rows": round(sum(x.numel() * 2 for x in streams) / 1e9, 1)},
        "roofline": None,
    }
    sv.close()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
