#!/usr/bin/env python3
"""Benchmark: all pairs within Levenshtein distance k among N CDR3-like
sequences by symmetric-deletion lookup on one MI355X.

One step = one sd_self_search call: pack, variant generation, grouping sort,
in-group pair emission, pair sort, verification and compaction, with the
input already resident in HBM and the result left in HBM. Prints one JSON
line. The CPU oracle is timed on a bounded sample of the same workload as a
reported baseline (single thread).
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
    "plain_10m_k1": ("plain_10m", 1),
    "plain_10m_k2": ("plain_10m", 2),
}
HBM_PEAK_GBS = 8000.0


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def cpu_baseline(codes, offsets, k, target_s=15.0):
    """The oracle, as it stands, on the first S sequences of the workload."""
    import cdr3gen
    import oracle
    n = 2000
    while True:  # grow the sample until one run takes about target_s
        c, o = cdr3gen.subset(codes, offsets, n)
        t0 = time.perf_counter()
        a, _, _ = oracle.self_search(c, o, k)
        dt = time.perf_counter() - t0
        if dt >= 0.5 * target_s or n >= len(offsets) - 1:
            break
        grow = min(8.0, max(1.5, target_s / max(dt, 1e-3)))
        n = min(len(offsets) - 1, int(n * grow))
    return {"value": len(a) / dt, "unit": "pairs/s", "cores": 1, "kind": "oracle",
            "sample": f"first {n} sequences of the workload, k={k}, one thread: "
                      f"{len(a)} pairs in {dt:.2f} s ({n / dt:.0f} sequences/s)",
            "seconds": dt, "sample_seqs": n, "sample_pairs": int(len(a))}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="plain_1m_k2", choices=sorted(WORKLOADS))
    ap.add_argument("--path", type=int, default=0, help="grouping path (0 auto, 1 full-key sort)")
    ap.add_argument("--group-cap", type=int, default=0, help="hashed path LDS capacity (0 auto)")
    ap.add_argument("--group-bits", type=int, default=0, help="hashed path hash bits (0 auto)")
    ap.add_argument("--sort-items", type=int, default=0, help="keys-only radix items/thread (0 auto)")
    ap.add_argument("--copy-calibration-mb", type=int, default=0,
                    help="run one device copy of this size first (a known-size kernel for counters)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--json-out", default=None)
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU only; --gpus must be 1", file=sys.stderr)
        sys.exit(2)

    import torch
    import cdr3gen
    from paper_2403_09010_amd import Context
    from paper_2403_09010_amd.symdel import (OPT_GROUP_BITS, OPT_GROUP_CAP, OPT_PATH,
                                             OPT_SORT_ITEMS, OPT_TIMING, _Seqs)

    gen_name, k = WORKLOADS[args.workload]
    log(f"generating {gen_name}")
    codes, offsets = cdr3gen.plain(gen_name)
    n = len(offsets) - 1
    dev = torch.device("cuda", 0)
    codes_t = torch.from_numpy(codes).to(dev)
    offs_t = torch.from_numpy(offsets).to(dev)
    seqs = _Seqs(codes_t.data_ptr(), offs_t.data_ptr(), n, 1)
    ctx = Context(0)
    ctx.set_option(OPT_PATH, args.path)
    ctx.set_option(OPT_GROUP_CAP, args.group_cap)
    ctx.set_option(OPT_GROUP_BITS, args.group_bits)
    ctx.set_option(OPT_SORT_ITEMS, args.sort_items)
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
        ctx.free_pairs(ctx.self_search_raw(seqs, k, sh))
    torch.cuda.synchronize()

    # timed region: K whole searches, stage events recorded on the same stream
    ctx.set_option(OPT_TIMING, 1)
    stage_ms, stage_bytes, stage_launch = {}, {}, {}
    npairs = None
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for step in range(args.steps):
        p = ctx.self_search_raw(seqs, k, sh)
        npairs = p.n
        ctx.free_pairs(p)
        st = ctx.stats()
        for s in st["stages"]:
            stage_ms[s["name"]] = stage_ms.get(s["name"], 0.0) + s["ms"]
            stage_bytes[s["name"]] = s["bytes"]
            stage_launch[s["name"]] = s["launches"]
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    st = ctx.stats()
    log(f"{args.workload}: {npairs} pairs, {dt * 1e3:.2f} ms/step, keys {st['n_keys']}, "
        f"raw candidates {st['n_cand_raw']}, sort passes {st['n_sort_passes']}")
    for name in stage_ms:
        ms = stage_ms[name] / args.steps
        gbs = stage_bytes[name] / (ms * 1e-3) / 1e9 if ms > 0 else 0.0
        log(f"  stage {name:12s} {ms:8.3f} ms  {stage_launch[name]:3d} launches  {gbs:8.1f} GB/s algorithmic")

    # dominant stage -> roofline entry (per-launch average)
    dom = max(stage_ms, key=lambda s: stage_ms[s])
    dom_ms = stage_ms[dom] / args.steps
    launches = max(1, stage_launch[dom])
    per_launch_bytes = stage_bytes[dom] / launches
    per_launch_s = dom_ms * 1e-3 / launches
    achieved = per_launch_bytes / per_launch_s / 1e9
    roofline = {"bound": "hbm", "kernel_stage": dom, "achieved": round(achieved, 1),
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": None, "launches_per_step": launches,
                "avg_launch_ms": round(per_launch_s * 1e3, 4),
                "algorithmic_bytes_per_launch": per_launch_bytes}
    value = npairs / dt
    out = {
        "metric": "End-to-end s & pairs/s, 1M CDR3 self-search k<=2 (pairs/s)",
        "value": round(value, 1), "unit": "pairs/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(dt * 1e3, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u128",
        "data": "synthetic (seeded CDR3-like generator)",
        "config": {"workload": args.workload, "n_seqs": n, "k": k, "seed": cdr3gen.PLAIN_CONFIGS[gen_name][0],
                   "pairs": int(npairs), "keys": st["n_keys"], "candidates_raw": st["n_cand_raw"],
                   "seconds_per_search": round(dt, 6), "path": args.path,
                   "group_cap": args.group_cap, "group_bits": args.group_bits,
                   "sort_items": args.sort_items},
        "stages_ms": {s: round(stage_ms[s] / args.steps, 4) for s in stage_ms},
        "roofline": roofline,
    }
    ctx.close()
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on a bounded sample")
        out["cpu_baseline"] = cpu_baseline(codes, offsets, k)
    line = json.dumps(out)
    print(line, flush=True)
    if args.json_out:
        with open(args.json_out, "w") as f:
            f.write(line + "\n")


if __name__ == "__main__":
    main()
