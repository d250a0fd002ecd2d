#!/usr/bin/env python3
"""Benchmark: all pairs within Levenshtein distance k among N CDR3-like
sequences by symmetric-deletion lookup on one MI355X.

One step = one sd_self_search call: pack, variant generation, grouping sort,
in-group pair emission, pair sort, verification and compaction, with the
input already resident in HBM and the result left in HBM (`value`). The
same search from host codes to host pairs (H2D and D2H included) is reported
beside it as `end_to_end`. Prints one JSON line. The CPU oracle is timed on
the host's cores as a reported baseline: the sharded oracle over the whole
workload where that fits the time bound (1M sequences, k=2), a bounded
prefix otherwise, and the single-thread oracle on a bounded prefix.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

WORKLOADS = {
    # name: (generator config, k)
    "plain_10k_k1": ("plain_10k", 1),
    "plain_1m_k2": ("plain_1m", 2),
    "plain_1m_k3": ("plain_1m", 3),
    "plain_10m_k1": ("plain_10m", 1),
    "plain_10m_k2": ("plain_10m", 2),
    "paired_1m_k2": ("paired_1m", 2),
}
# paired-chain records: seed and count of cdr3gen.paired
PAIRED_CONFIGS = {"paired_1m": (9, 1_000_000)}
HBM_PEAK_GBS = 8000.0
# HBM bytes per launch from the FETCH_SIZE and WRITE_SIZE counters, scaled by a
# 1 GiB copy (profiles/traffic_hashed_path_plain_1m_k2.md), for the stages and
# workload they were taken on; other stages and workloads report null. They
# are a stored profile, not a measurement of this run: TRAFFIC_SOURCE names it.
# (both hash passes run over the same fixed tiles, so the counters give one
# mean over their 14 dispatches)
TRAFFIC_PER_LAUNCH = {("plain_1m_k2", "hash_counted_pass"): 1.6594e9,
                      ("plain_1m_k2", "hash_passes"): 1.6594e9}
TRAFFIC_SOURCE = ("rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE of k_scatter_counted, "
                  "profiles/traffic_hashed_path_plain_1m_k2.md (kernel and tiles unchanged since)")
# method floor of the end-to-end fraction: every deletion variant written once,
# read and written by one grouping pass and read once more (20-byte key records)
E2E_BYTES_PER_KEY = 80
METRICS = {
    "plain_10k_k1": "End-to-end s & pairs/s, 10K CDR3 self-search k<=1 (pairs/s)",
    "plain_1m_k2": "End-to-end s & pairs/s, 1M CDR3 self-search k<=2 (pairs/s)",
    "plain_10m_k1": "End-to-end s & pairs/s, 10M CDR3 self-search k<=1 (pairs/s)",
    "plain_10m_k2": "End-to-end s & pairs/s, 10M CDR3 self-search k<=2 (pairs/s)",
    "plain_1m_k3": "End-to-end s & pairs/s, 1M CDR3 self-search k<=3 (pairs/s)",
    "paired_1m_k2": "End-to-end s & pairs/s, 1M paired-chain records, Lev(a)+Lev(b)<=2 (pairs/s)",
}
# stages that time exactly one kernel (launched once, or several times alike)
KERNEL_OF_STAGE = {
    "vargen_hash": "k_vargen_hash",
    "hash_passes": "k_scatter_counted",
    "hash_counted_pass": "k_scatter_counted",
    "verify": "k_verify_compact",
    "sort_passes": "k_onesweep",
    "emit": "k_emit_runs",
}
HBM_STAGES = ("hash_passes", "hash_counted_pass", "sort_passes")


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(codes, offsets, k, target_s=15.0, threads=1, paired=None):
    """The oracle, as it stands, on the first S sequences (or records) of the
    workload (S grown until one run takes about target_s); threads > 1 runs the
    sharded oracle on that many threads. paired: the second chains (codes,
    offsets) of paired-chain records (the oracle's paired mode, one thread)."""
    import cdr3gen
    import oracle
    n = 2000
    while True:  # grow the sample until one run takes about target_s
        c, o = cdr3gen.subset(codes, offsets, n)
        t0 = time.perf_counter()
        if paired is not None:
            a, _, _ = oracle.paired_self_search((c, o), cdr3gen.subset(*paired, n), k)
        elif threads > 1:
            a, _, _ = oracle.self_search_sharded(c, o, k, threads=threads)
        else:
            a, _, _ = oracle.self_search(c, o, k)
        dt = time.perf_counter() - t0
        if dt >= 0.5 * target_s or n >= len(offsets) - 1:
            break
        grow = min(8.0, max(1.5, target_s / max(dt, 1e-3)))
        n = min(len(offsets) - 1, int(n * grow))
    whole = n >= len(offsets) - 1
    unit = "records" if paired is not None else "sequences"
    what = "the whole workload" if whole else f"first {n} {unit} of the workload"
    mode = ("paired-chain oracle on one thread" if paired is not None else
            f"sharded oracle on {threads} threads" if threads > 1 else "oracle on one thread")
    return {"value": len(a) / dt, "unit": "pairs/s", "cores": threads, "kind": "oracle",
            "sample": f"{what}, k={k}, {mode}: {len(a)} pairs in {dt:.2f} s "
                      f"({n / dt:.0f} sequences/s)",
            "seconds": dt, "sample_seqs": n, "sample_pairs": int(len(a)), "whole_workload": whole,
            "host_cpu": cpu_model(), "host_nproc": os.cpu_count()}


def cpu_baselines(codes, offsets, k, workload, paired=None):
    """The sharded oracle on the host's cores (the whole 1M workload fits the
    bound: about 20-35 s), plus the single-thread oracle on a bounded prefix."""
    import oracle
    threads = oracle.host_threads()
    if workload.startswith("paired"):
        one = cpu_baseline(codes, offsets, k, target_s=15.0, threads=1, paired=paired)
        return one, one
    if workload in ("plain_1m_k2", "plain_10k_k1"):
        t0 = time.perf_counter()
        a, _, _ = oracle.self_search_sharded(codes, offsets, k, threads=threads)
        dt = time.perf_counter() - t0
        n = len(offsets) - 1
        allc = {"value": len(a) / dt, "unit": "pairs/s", "cores": threads, "kind": "oracle",
                "sample": f"the whole workload ({n} sequences), k={k}, sharded oracle on "
                          f"{threads} threads: {len(a)} pairs in {dt:.2f} s",
                "seconds": dt, "sample_seqs": n, "sample_pairs": int(len(a)),
                "whole_workload": True, "host_cpu": cpu_model(), "host_nproc": os.cpu_count()}
    else:
        allc = cpu_baseline(codes, offsets, k, target_s=20.0, threads=threads)
    one = cpu_baseline(codes, offsets, k, target_s=10.0, threads=1)
    return allc, one


def emit(out, args):
    line = json.dumps(out)
    print(line, flush=True)
    if args.json_out:
        with open(args.json_out, "w") as f:
            f.write(line + "\n")


def run_batched(args):
    """512 query sets against one 2M-sequence reference index at k=2: one set
    per launch (sd_query) versus all sets in one batched call (sd_query_batch),
    eagerly in tiles and as one captured HIP graph (captured in the warm-up,
    replayed in the timed steps)."""
    import torch
    import cdr3gen
    from paper_2403_09010_amd import Context
    from paper_2403_09010_amd.symdel import OPT_BATCH_GRAPH, _Seqs
    p = cdr3gen.BATCHED
    k = 2
    nsets = args.sets
    log(f"generating the {p['ref_n']}-sequence reference and {nsets} query sets")
    ref = cdr3gen.generate(p["ref_seed"], p["ref_n"])
    sets = cdr3gen.batched_sets(ref, nsets, args.set_scale)
    nq = sum(len(o) - 1 for _, o in sets)
    dev = torch.device("cuda", 0)
    ctx = Context(0)
    stream = int(torch.cuda.current_stream().cuda_stream)
    t0 = time.perf_counter()
    idx = ctx.build_index(torch.from_numpy(ref[0]).to(dev), torch.from_numpy(ref[1]).to(dev), k)
    torch.cuda.synchronize()
    t_index = time.perf_counter() - t0
    info = idx.info()
    log(f"index: {info} in {t_index:.2f} s; {nq} query sequences")
    dsets = [(torch.from_numpy(c).to(dev), torch.from_numpy(o).to(dev)) for c, o in sets]
    tune = None
    if not args.no_autotune:
        # tile size and radix items per thread from the autotuner, on these sets
        tune = ctx.autotune(dsets, k, index=idx, reps=1)
        log(f"autotune: {tune}")
    arr = (_Seqs * nsets)()
    for x, (c, o) in enumerate(dsets):
        arr[x] = _Seqs(c.data_ptr() if c.numel() else None, o.data_ptr(), o.numel() - 1, 1)

    def plain_once():
        tot = 0
        for x in range(nsets):
            outs = ctx.query_batch_raw(idx, ctypes_pointer(arr, x), 1, k, stream)
            tot += outs[0].n
            ctx.free_pairs(outs[0])
        return tot

    def batched_once():
        outs = ctx.query_batch_raw(idx, arr, nsets, k, stream)
        tot = sum(outs[x].n for x in range(nsets))
        for x in range(nsets):
            ctx.free_pairs(outs[x])
        return tot

    res = {}
    graph_stats = None
    modes = [m for m in ("plain", "batched", "graph") if m in args.batched_modes.split(",")]
    assert modes, "--batched-modes names none of plain, batched, graph"
    fns = {"plain": plain_once, "batched": batched_once, "graph": batched_once}
    for name in modes:
        fn = fns[name]
        ctx.set_option(OPT_BATCH_GRAPH, 1 if name == "graph" else 0)
        for _ in range(args.warmup):
            fn()
        if name == "graph":
            # the first calls capture, and the capacity may settle once (one
            # more capture): warm up until a call replays
            for _ in range(4):
                fn()
                if ctx.stats()["n_graph_captures"] == 0:
                    break
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            pairs = fn()
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / args.steps
        res[name] = (dt, pairs)
        if name == "graph":
            graph_stats = {x: ctx.stats()[x] for x in ("n_graph_captures", "n_graph_launches",
                                                       "n_graph_retries")}
        log(f"{name}: {dt * 1e3:.1f} ms per run, {pairs} pairs")
    ctx.set_option(OPT_BATCH_GRAPH, 0)
    assert len({res[m][1] for m in modes}) == 1, {m: res[m][1] for m in modes}
    head = modes[-1]  # the graph if timed, else the eager batch
    dt, pairs = res[head]

    def mode_rec(m):
        if m not in res:
            return None
        return {"seconds": round(res[m][0], 4), "pairs_per_s": round(res[m][1] / res[m][0], 1)}

    def ratio(a, b):
        return round(res[a][0] / res[b][0], 3) if a in res and b in res else None
    out = {
        "metric": "Batched query: 512 repertoires vs 2M reference, k=2 (pairs/s)",
        "value": round(pairs / dt, 1), "unit": "pairs/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(dt * 1e3, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u64",
        "data": "synthetic (seeded CDR3-like generator)",
        "config": {"workload": "batched_2m_512", "ref_n": p["ref_n"], "sets": nsets,
                   "query_seqs": nq, "k": k, "pairs": int(pairs),
                   "index_keys": info["n_keys"], "index_build_s": round(t_index, 3)},
        "plain_one_set_per_launch": mode_rec("plain"),
        "batched_tiles": mode_rec("batched"),
        "graph": dict(mode_rec("graph"), last_call=graph_stats) if "graph" in res else None,
        "value_is": {"graph": "pairs / seconds of one sd_query_batch call as a replayed captured graph",
                     "batched": "pairs / seconds of one sd_query_batch call (eager tiles)",
                     "plain": "pairs / seconds of 512 sd_query calls, one set each"}[head],
        "speedup_graph_vs_plain": ratio("plain", "graph"),
        "speedup_graph_vs_tiles": ratio("batched", "graph"),
        "speedup_tiles_vs_plain": ratio("plain", "batched"),
        "autotune": tune,
    }
    idx.free()
    ctx.close()
    emit(out, args)


def ctypes_pointer(arr, x):
    import ctypes
    from paper_2403_09010_amd.symdel import _Seqs
    return ctypes.cast(ctypes.byref(arr, x * ctypes.sizeof(_Seqs)), ctypes.POINTER(_Seqs))


def run_served(args):
    """Poisson-arriving query sets (sizes log-uniform in [100, 5e4]) against a
    5M-sequence reference index, weighted rescoring (costs {3, 4}, indel 8,
    score <= 8), continuous batching versus one request at a time."""
    import threading
    import torch
    import cdr3gen
    from paper_2403_09010_amd import Context, Server
    p = cdr3gen.SERVED
    log(f"generating the {p['ref_n'] // args.ref_div}-sequence reference")
    ref = cdr3gen.generate(p["ref_seed"], p["ref_n"] // args.ref_div)
    dev = torch.device("cuda", 0)
    ctx = Context(0)
    t0 = time.perf_counter()
    idx = ctx.build_index(torch.from_numpy(ref[0]).to(dev), torch.from_numpy(ref[1]).to(dev), 2)
    torch.cuda.synchronize()
    t_index = time.perf_counter() - t0
    info = idx.info()
    log(f"index: {info} in {t_index:.2f} s")
    subst = cdr3gen.cost_matrix(p["cost_seed"], p["cost_lo"], p["cost_hi"])
    nreq = args.requests
    sizes = cdr3gen.loguniform_sizes(p["arrival_seed"], nreq, p["size_lo"], p["size_hi"])
    reqs = [cdr3gen.generate_query(20000 + x, int(n), *ref, ref_mut_frac=0.1)
            for x, n in enumerate(sizes)]

    def run(server_kw, rate, count):
        """Submit `count` requests (rate None: all at once); return latencies, wall time, pairs."""
        with Server(idx, k=2, subst=subst, indel=p["indel"], max_score=p["max_score"],
                    **server_kw) as sv:
            ids = [None] * count
            t_arr = (cdr3gen.poisson_arrivals(p["arrival_seed"], count, rate)
                     if rate else np.zeros(count))
            start = time.perf_counter()

            def producer():
                for x in range(count):
                    wait = start + t_arr[x] - time.perf_counter()
                    if wait > 0:
                        time.sleep(wait)
                    ids[x] = sv.submit(*reqs[x % nreq])

            th = threading.Thread(target=producer)
            th.start()
            lats, pairs = [], 0
            for x in range(count):
                while ids[x] is None:
                    time.sleep(0.0002)
                r, lat = sv.poll(ids[x], timeout_ms=600000)
                lats.append(lat)
                pairs += len(r)
            th.join()
            wall = time.perf_counter() - start
            st = sv.stats()
        return np.array(lats), wall, pairs, st

    # saturation throughput X: everything queued at once
    burst = min(nreq, args.burst)
    lats, wall, pairs, st = run({"workers": 2}, None, burst)
    X = burst / wall
    log(f"saturation: {burst} requests in {wall:.2f} s -> X = {X:.1f} req/s, batches {st}")
    _, wall1, _, st1 = run({"workers": 1, "max_batch_requests": 1}, None, min(burst, 200))
    X1 = min(burst, 200) / wall1
    log(f"serial saturation: {X1:.1f} req/s")
    rates = {}
    for frac in (0.5, 0.9):
        rate = frac * X
        lats, wall, pairs, st = run({"workers": 2}, rate, nreq)
        rates[str(frac)] = {"rate_req_s": round(rate, 2), "p50_ms": round(np.percentile(lats, 50) * 1e3, 2),
                            "p99_ms": round(np.percentile(lats, 99) * 1e3, 2),
                            "throughput_req_s": round(nreq / wall, 2),
                            "pairs_per_s": round(pairs / wall, 1), "batches": st["batches"],
                            "max_batch": st["max_batch"]}
        log(f"rate {rate:.1f}/s: {rates[str(frac)]}")
        lats_s, wall_s, _, _ = run({"workers": 1, "max_batch_requests": 1}, rate,
                                   min(nreq, args.serial_requests))
        rates[str(frac)]["serial_p50_ms"] = round(np.percentile(lats_s, 50) * 1e3, 2)
        rates[str(frac)]["serial_p99_ms"] = round(np.percentile(lats_s, 99) * 1e3, 2)
        log(f"  serial at the same rate: p50 {rates[str(frac)]['serial_p50_ms']} ms, "
            f"p99 {rates[str(frac)]['serial_p99_ms']} ms")
    # one request alone through the context (host set in, host result out):
    # a 3,000-sequence set, median of 20 after 3 warm-up calls
    one = cdr3gen.generate_query(29999, 3000, *ref, ref_mut_frac=0.1)
    for _ in range(3):
        ctx.query_weighted(idx, *one, subst, p["indel"], p["max_score"], device_output=False)
    t_one = []
    for _ in range(20):
        t1 = time.perf_counter()
        ctx.query_weighted(idx, *one, subst, p["indel"], p["max_score"], device_output=False)
        t_one.append(time.perf_counter() - t1)
    single = {"seqs": 3000, "ms_median_of_20": round(float(np.median(t_one)) * 1e3, 3)}
    log(f"one 3,000-sequence request alone: {single['ms_median_of_20']} ms")
    out = {
        "metric": "Served: Poisson query sets vs 5M reference, weighted score <= 8 (requests/s)",
        "value": round(X, 2), "unit": "requests/s", "n_gpus": 1, "steps": nreq, "warmup": 0,
        "ms_per_step": round(1e3 / X, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u64", "data": "synthetic (seeded CDR3-like generator)",
        "config": {"workload": "served_5m", "ref_n": int(len(ref[1]) - 1), "requests": nreq,
                   "index_keys": info["n_keys"], "index_build_s": round(t_index, 3),
                   "saturation_req_s": round(X, 2), "serial_saturation_req_s": round(X1, 2)},
        "poisson": rates,
        "single_request": single,
    }
    idx.free()
    ctx.close()
    emit(out, args)


def run_learned(args):
    """The learned reference index against its own lookup without the model:
    one query set against the 5M-sequence reference at k=2, probe stage timed
    with the model's window (probe 0) and with a binary search over the whole
    sorted key array (probe 1); the hashed index is timed beside them."""
    import torch
    import cdr3gen
    from paper_2403_09010_amd import Context, OPT_PROBE, OPT_TIMING
    p = cdr3gen.SERVED
    k = 2
    log(f"generating the {p['ref_n'] // args.ref_div}-sequence reference")
    ref = cdr3gen.generate(p["ref_seed"], p["ref_n"] // args.ref_div)
    qry = cdr3gen.generate_query(30000, args.learned_queries, *ref, ref_mut_frac=0.1)
    dev = torch.device("cuda", 0)
    ctx = Context(0)
    rd = (torch.from_numpy(ref[0]).to(dev), torch.from_numpy(ref[1]).to(dev))
    qd = (torch.from_numpy(qry[0]).to(dev), torch.from_numpy(qry[1]).to(dev))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lidx = ctx.build_learned_index(*rd, k, leaves_log2=args.leaves_log2)
    torch.cuda.synchronize()
    t_learned = time.perf_counter() - t0
    info = lidx.learned_info()
    log(f"learned index: {lidx.info()} in {t_learned:.2f} s; leaves {info['leaves']}, "
        f"mean eps {info['mean_eps']:.1f}, max eps {info['max_eps']}, mean window log2 "
        f"{info['mean_window_log2']:.2f}, loss {info['loss_first']:.3g} -> {info['loss_last']:.3g}, "
        f"train {info['train_ms']:.1f} ms, fit {info['fit_ms']:.1f} ms")
    t0 = time.perf_counter()
    hidx = ctx.build_index(*rd, k)
    torch.cuda.synchronize()
    t_hashed = time.perf_counter() - t0
    ctx.set_option(OPT_TIMING, 1)
    res = {}
    for name, idx, probe in (("learned", lidx, 0), ("binary", lidx, 1), ("hashed", hidx, 0)):
        ctx.set_option(OPT_PROBE, probe)
        for _ in range(args.warmup):
            ctx.query(idx, *qd, k)
        torch.cuda.synchronize()
        stage, tot, steps = {}, 0.0, 0
        t0 = time.perf_counter()
        for _ in range(args.steps):
            r = ctx.query(idx, *qd, k)
            st = ctx.stats()
            for sg in st["stages"]:
                stage[sg["name"]] = stage.get(sg["name"], 0.0) + sg["ms"] / args.steps
            steps = st["n_probe_steps"]
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / args.steps
        res[name] = {"seconds": round(dt, 5), "pairs": len(r), "query_keys": st["n_keys"],
                     "candidates": st["n_cand_raw"],
                     "comparisons_per_lookup": round(steps / max(1, st["n_keys"]), 3),
                     "stages_ms": {a: round(b, 4) for a, b in stage.items()}}
        log(f"{name}: {res[name]}")
    assert res["learned"]["pairs"] == res["binary"]["pairs"] == res["hashed"]["pairs"]
    lp = res["learned"]["stages_ms"].get("probe", 0.0)
    bp = res["binary"]["stages_ms"].get("probe", 0.0)
    nkeys = res["learned"]["query_keys"]
    out = {
        "metric": "Learned index: query-key lookups/s in the probe stage, 5M reference k=2",
        "value": round(nkeys / (lp * 1e-3), 1) if lp else None, "unit": "lookups/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(res["learned"]["seconds"] * 1e3, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32 model, u128 keys",
        "data": "synthetic (seeded CDR3-like generator)",
        "config": {"workload": "learned_5m", "ref_n": int(len(ref[1]) - 1),
                   "query_seqs": args.learned_queries, "k": k, "index_keys": lidx.info()["n_keys"],
                   "leaves": info["leaves"], "learned_build_s": round(t_learned, 3),
                   "hashed_build_s": round(t_hashed, 3)},
        "model": {"mean_eps": round(info["mean_eps"], 2), "max_eps": int(info["max_eps"]),
                  "mean_window_log2": round(info["mean_window_log2"], 3),
                  "empty_leaves": int(info["empty_leaves"]), "steps": int(info["steps"]),
                  "loss_first": float(info["loss_first"]), "loss_last": float(info["loss_last"]),
                  "train_ms": round(info["train_ms"], 2), "fit_ms": round(info["fit_ms"], 2)},
        "learned": res["learned"], "binary_search": res["binary"], "hashed_index": res["hashed"],
        "probe_speedup_learned_vs_binary": round(bp / lp, 3) if lp else None,
    }
    lidx.free()
    hidx.free()
    ctx.close()
    emit(out, args)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="plain_1m_k2",
                    choices=sorted(WORKLOADS) + ["batched_2m_512", "served_5m", "learned_5m"])
    ap.add_argument("--sets", type=int, default=512, help="batched: number of query sets")
    ap.add_argument("--set-scale", type=float, default=1.0, help="batched: scale of set sizes")
    ap.add_argument("--requests", type=int, default=2000, help="served: requests per rate")
    ap.add_argument("--burst", type=int, default=2000, help="served: requests for saturation")
    ap.add_argument("--serial-requests", type=int, default=200, help="served: serial comparison")
    ap.add_argument("--ref-div", type=int, default=1, help="served/learned: reference size divisor")
    ap.add_argument("--learned-queries", type=int, default=200000, help="learned: query sequences")
    ap.add_argument("--leaves-log2", type=int, default=0, help="learned: leaves (0 automatic)")
    ap.add_argument("--path", type=int, default=0, help="grouping path (0 auto, 1 full-key sort)")
    ap.add_argument("--group-cap", type=int, default=0, help="hashed path LDS capacity (0 auto)")
    ap.add_argument("--group-bits", type=int, default=0, help="hashed path hash bits (0 auto)")
    ap.add_argument("--sort-items", type=int, default=0, help="keys-only radix items/thread (0 auto)")
    ap.add_argument("--group-batches", type=int, default=0, help="hashed path LDS batches per workgroup (0 auto)")
    ap.add_argument("--group-shape", type=int, default=0, help="grouping kernel shape at capacity 2048 (0-2)")
    ap.add_argument("--budget-gb", type=float, default=0.0,
                    help="device memory budget of the context in GiB (0: none); a search "
                         "that does not fit streams in column groups")
    ap.add_argument("--pair-sort", type=int, default=0,
                    help="candidate pair sort (0 auto: bucketed in LDS, 1 one-sweep, 2 counted)")
    ap.add_argument("--batched-modes", default="plain,batched,graph",
                    help="batched: which of plain, batched, graph to time")
    ap.add_argument("--stream", type=int, default=0, help="streamed search: 0 auto, 1 never, 2 always")
    ap.add_argument("--stream-elems", type=int, default=0, help="streamed search: variants per group (0 auto)")
    ap.add_argument("--copy-calibration-mb", type=int, default=0,
                    help="run one device copy of this size first (a known-size kernel for counters)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true", help="batched: keep the default options")
    ap.add_argument("--json-out", default=None)
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: the search runs on one GPU; --gpus must be 1", file=sys.stderr)
        sys.exit(2)
    if args.workload == "batched_2m_512":
        return run_batched(args)
    if args.workload == "served_5m":
        return run_served(args)
    if args.workload == "learned_5m":
        return run_learned(args)

    import torch
    import cdr3gen
    from paper_2403_09010_amd import Context
    from paper_2403_09010_amd.symdel import (OPT_GROUP_BATCHES, OPT_GROUP_BITS, OPT_GROUP_CAP,
                                             OPT_GROUP_SHAPE, OPT_PAIR_SORT, OPT_PATH,
                                             OPT_SORT_ITEMS, OPT_STREAM, OPT_STREAM_ELEMS,
                                             OPT_TIMING, _Seqs)

    gen_name, k = WORKLOADS[args.workload]
    log(f"generating {gen_name}")
    paired = gen_name in PAIRED_CONFIGS
    chain_b = None
    if paired:
        seed = PAIRED_CONFIGS[gen_name][0]
        (codes, offsets), chain_b = cdr3gen.paired(*PAIRED_CONFIGS[gen_name])
    else:
        seed = cdr3gen.PLAIN_CONFIGS[gen_name][0]
        codes, offsets = cdr3gen.plain(gen_name)
    n = len(offsets) - 1
    dev = torch.device("cuda", 0)
    codes_t = torch.from_numpy(codes).to(dev)
    offs_t = torch.from_numpy(offsets).to(dev)
    seqs = _Seqs(codes_t.data_ptr(), offs_t.data_ptr(), n, 1)
    seqs_b = None
    if paired:
        codes_bt = torch.from_numpy(chain_b[0]).to(dev)
        offs_bt = torch.from_numpy(chain_b[1]).to(dev)
        seqs_b = _Seqs(codes_bt.data_ptr(), offs_bt.data_ptr(), n, 1)
    ctx = Context(0, hbm_budget=int(args.budget_gb * (1 << 30)))
    ctx.set_option(OPT_PATH, args.path)
    ctx.set_option(OPT_GROUP_CAP, args.group_cap)
    ctx.set_option(OPT_GROUP_BITS, args.group_bits)
    ctx.set_option(OPT_SORT_ITEMS, args.sort_items)
    ctx.set_option(OPT_GROUP_BATCHES, args.group_batches)
    ctx.set_option(OPT_GROUP_SHAPE, args.group_shape)
    ctx.set_option(OPT_PAIR_SORT, args.pair_sort)
    ctx.set_option(OPT_STREAM, args.stream)
    ctx.set_option(OPT_STREAM_ELEMS, args.stream_elems)

    def search_raw():
        if paired:
            return ctx.paired_self_search_raw(seqs, seqs_b, k, sh)

        return ctx.self_search_raw(seqs, k, sh)

    def search_host():
        if paired:
            return ctx.paired_self_search((codes, offsets), chain_b, k, device_output=False)
        return ctx.self_search(codes, offsets, k, device_output=False)
    if args.copy_calibration_mb:
        src = torch.empty(args.copy_calibration_mb << 20, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    stream = torch.cuda.current_stream()
    sh = int(stream.cuda_stream)

    log(f"warmup {args.warmup}")
    for _ in range(args.warmup):
        ctx.free_pairs(search_raw())
    torch.cuda.synchronize()

    # timed region: K whole searches, stage events recorded on the same stream
    ctx.set_option(OPT_TIMING, 1)
    stage_ms, stage_bytes, stage_launch = {}, {}, {}
    npairs = None
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for step in range(args.steps):
        p = search_raw()
        npairs = p.n
        ctx.free_pairs(p)
        st = ctx.stats()
        # a stage name can repeat within a search (one mark per pass): its
        # bytes and launches per search are the sums over its marks
        step_bytes, step_launch = {}, {}
        for s in st["stages"]:
            stage_ms[s["name"]] = stage_ms.get(s["name"], 0.0) + s["ms"]
            step_bytes[s["name"]] = step_bytes.get(s["name"], 0.0) + s["bytes"]
            step_launch[s["name"]] = step_launch.get(s["name"], 0) + s["launches"]
        stage_bytes.update(step_bytes)
        stage_launch.update(step_launch)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    st = ctx.stats()
    log(f"{args.workload}: {npairs} pairs, {dt * 1e3:.2f} ms/step, keys {st['n_keys']}, "
        f"raw candidates {st['n_cand_raw']}, sort passes {st['n_sort_passes']}")
    for name in stage_ms:
        ms = stage_ms[name] / args.steps
        gbs = stage_bytes[name] / (ms * 1e-3) / 1e9 if ms > 0 else 0.0
        log(f"  stage {name:12s} {ms:8.3f} ms  {stage_launch[name]:3d} launches  {gbs:8.1f} GB/s algorithmic")

    # host-to-host: u8 codes and offsets in host memory, pairs back in host
    # memory (H2D and D2H included); one warm-up, median of five
    ctx.set_option(OPT_TIMING, 0)
    search_host()
    h2h = []
    for _ in range(5):
        t1 = time.perf_counter()
        r = search_host()
        h2h.append(time.perf_counter() - t1)
    h2h_s = float(np.median(h2h))
    assert len(r) == npairs
    log(f"host-to-host: {h2h_s * 1e3:.2f} ms median of 5")

    # roofline entries: the dominant single-kernel stage, and the LSD sort
    # passes; per-launch algorithmic bytes over the per-launch device time
    def roof(stage):
        ms = stage_ms[stage] / args.steps
        launches = max(1, stage_launch[stage])
        per_launch_bytes = stage_bytes[stage] / launches
        per_launch_s = ms * 1e-3 / launches
        achieved = per_launch_bytes / per_launch_s / 1e9
        traffic = TRAFFIC_PER_LAUNCH.get((args.workload, stage))
        if (args.path or args.group_cap or args.group_bits or args.sort_items or args.group_batches
                or args.group_shape or args.budget_gb or args.stream or args.pair_sort):
            traffic = None  # the counters were taken with the default configuration
        return {"bound": "hbm", "kernel": KERNEL_OF_STAGE[stage], "stage": stage,
                "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "traffic_source": TRAFFIC_SOURCE if traffic is not None else None,
                "launches_per_step": launches, "avg_launch_ms": round(per_launch_s * 1e3, 4),
                "algorithmic_bytes_per_launch": per_launch_bytes}

    single = [x for x in stage_ms if x in KERNEL_OF_STAGE and stage_launch[x] > 0]
    # the dominant HBM-bound kernel (variant generation is ALU-bound, the
    # grouping LDS/latency-bound; their stage times are in stages_ms)
    hbm = [x for x in single if x in HBM_STAGES] or single
    dom = max(hbm, key=lambda x: stage_ms[x] / max(1, stage_launch[x]))
    roofline = roof(dom)
    sort_stage = "hash_passes" if "hash_passes" in single else "sort_passes"
    sort_roofline = roof(sort_stage) if sort_stage in single else None
    counted_roofline = roof("hash_counted_pass") if "hash_counted_pass" in single else None
    value = npairs / dt
    # end-to-end roofline fraction: the method floor (80 B per deletion
    # variant) over the measured time, against 8 TB/s
    nkeys = st["n_keys"]
    floor_bytes = E2E_BYTES_PER_KEY * nkeys
    out = {
        "metric": METRICS[args.workload],
        "value": round(value, 1), "unit": "pairs/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(dt * 1e3, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u128",
        "data": "synthetic (seeded CDR3-like generator)",
        "config": {"workload": args.workload, "n_seqs": n, "k": k, "seed": seed,
                   "pairs": int(npairs), "keys": st["n_keys"], "candidates_raw": st["n_cand_raw"],
                   "seconds_per_search": round(dt, 6), "path": args.path,
                   "group_cap": args.group_cap, "group_bits": args.group_bits,
                   "sort_items": args.sort_items, "group_batches": args.group_batches,
                   "group_shape": args.group_shape, "pair_sort": args.pair_sort,
                   "pair_buckets": st["n_pair_buckets"], "budget_gb": args.budget_gb,
                   "stream": args.stream, "stream_groups": st["n_stream_groups"]},
        "stages_ms": {s: round(stage_ms[s] / args.steps, 4) for s in stage_ms},
        "value_is": "pairs / device time of one search, inputs resident in HBM, result left in HBM",
        "end_to_end": {"seconds_median_of_5": round(h2h_s, 6),
                       "pairs_per_s": round(npairs / h2h_s, 1),
                       "what": "host u8 codes and offsets in, host (i, j, d) arrays out "
                               "(H2D and D2H over PCIe included)",
                       "frac": round(floor_bytes / h2h_s / (HBM_PEAK_GBS * 1e9), 4),
                       "device_resident_frac": round(floor_bytes / dt / (HBM_PEAK_GBS * 1e9), 4),
                       "frac_basis": f"{E2E_BYTES_PER_KEY} B x {nkeys} distinct deletion variants "
                                     f"(method floor) / time / 8 TB/s"},
        "roofline": roofline,
        "sort_roofline": sort_roofline,
        "counted_pass_roofline": counted_roofline,
    }
    ctx.close()
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on the host cores")
        allc, one = cpu_baselines(codes, offsets, k, args.workload, paired=chain_b)
        out["cpu_baseline"] = allc
        out["cpu_baseline_one_thread"] = one
        log(f"cpu baseline: {allc['sample']}; {one['sample']}")
    line = json.dumps(out)
    print(line, flush=True)
    if args.json_out:
        with open(args.json_out, "w") as f:
            f.write(line + "\n")


if __name__ == "__main__":
    main()
