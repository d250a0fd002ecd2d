"""Writes tests/golden/oracle_results.json from the CPU oracle only.

Run from the repository root:
    python tests/golden/make_golden.py                 # every entry except the 10M k=2 one
    python tests/golden/make_golden.py --only oracle_plain_10m_k2
The stored values are the generator's byte hashes (regression pins of the
input recipe) and the oracle's pair counts and pair-list hashes; nothing here
comes from the GPU library. The full-size entries use the oracle's sharded
mode, which the CPU pins hold equal to brute force and to the single-thread
oracle. Entries not named by --only keep their stored values.

A full-size entry also stores `chunk_sha256`: the hash of the triplets whose
first index lies in each of CHUNKS equal ranges of sequence ids, so that a
mismatch can be narrowed to one range without running the oracle again.
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import cdr3gen  # noqa: E402
import oracle  # noqa: E402

PATH = os.path.join(ROOT, "tests", "golden", "oracle_results.json")
CHUNKS = 16


def sha(*arrays):
    h = hashlib.sha256()
    for a in arrays:
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()


def triplet_entry(a, b, d, n=None):
    """Pair count and hash of (a u32, b u32, d u8); with n, per-range chunk hashes too."""
    d8 = d.astype(np.uint8)
    out = {"pairs": int(len(a)), "sha256": sha(a, b, d8)}
    if n is not None:
        edges = np.searchsorted(a, [n * x // CHUNKS for x in range(CHUNKS + 1)])
        out["chunk_sha256"] = [sha(a[lo:hi], b[lo:hi], d8[lo:hi]) for lo, hi in zip(edges[:-1], edges[1:])]
    return out


def entries():
    """name -> function computing the entry (lazily: some take minutes)."""
    def gen_sha(cfg):
        return lambda: sha(*cdr3gen.plain(cfg))

    def small(k):
        def f():
            c, o = cdr3gen.plain("plain_10k")
            return triplet_entry(*oracle.self_search(c, o, k))
        return f

    def prefix20k():
        cs, os_ = cdr3gen.subset(*cdr3gen.plain("plain_1m"), 20000)
        return triplet_entry(*oracle.self_search(cs, os_, 2))

    def full(cfg, k, shards):
        def f():
            c, o = cdr3gen.plain(cfg)
            t0 = time.time()
            a, b, d = oracle.self_search_sharded(c, o, k, shards=shards)
            print(f"{cfg} k={k}: {len(a)} pairs in {time.time() - t0:.1f} s", file=sys.stderr)
            return triplet_entry(a, b, d, n=len(o) - 1)
        return f

    return {
        "gen_plain_10k_sha256": gen_sha("plain_10k"),
        "gen_plain_1m_sha256": gen_sha("plain_1m"),
        "gen_plain_10m_sha256": gen_sha("plain_10m"),
        "oracle_plain_10k_k0": small(0),
        "oracle_plain_10k_k1": small(1),
        "oracle_plain_10k_k2": small(2),
        "oracle_plain_1m_first20k_k2": prefix20k,
        "oracle_plain_1m_k2": full("plain_1m", 2, 0),
        "oracle_plain_10m_k1": full("plain_10m", 1, 16),
        "oracle_plain_10m_k2": full("plain_10m", 2, 64),
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--only", nargs="*", default=None, help="entries to (re)compute")
    args = ap.parse_args()
    table = entries()
    names = args.only if args.only else [x for x in table if x != "oracle_plain_10m_k2"]
    out = json.load(open(PATH)) if os.path.exists(PATH) else {}
    for name in names:
        out[name] = table[name]()
        with open(PATH, "w") as f:  # written after every entry: long runs keep what they finished
            json.dump(out, f, indent=1, sort_keys=True)
    print(json.dumps({x: out[x] for x in names}, indent=1)[:4000])


if __name__ == "__main__":
    main()
