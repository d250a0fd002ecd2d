"""Writes tests/golden/oracle_results.json from the CPU oracle only.

Run from the repository root:  python tests/golden/make_golden.py
The stored values are the generator's byte hashes (regression pins of the
input recipe) and the oracle's pair counts and pair-list hashes for the
small workloads; nothing here comes from the GPU library.
"""
import hashlib
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import cdr3gen  # noqa: E402
import oracle  # noqa: E402


def sha(*arrays):
    h = hashlib.sha256()
    for a in arrays:
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()


def main():
    out = {}
    c, o = cdr3gen.plain("plain_10k")
    out["gen_plain_10k_sha256"] = sha(c, o)
    c1, o1 = cdr3gen.plain("plain_1m")
    out["gen_plain_1m_sha256"] = sha(c1, o1)
    for k in (0, 1, 2):
        a, b, d = oracle.self_search(c, o, k)
        out[f"oracle_plain_10k_k{k}"] = {"pairs": int(len(a)), "sha256": sha(a, b, d.astype(np.uint8))}
    cs, os_ = cdr3gen.subset(c1, o1, 20000)
    a, b, d = oracle.self_search(cs, os_, 2)
    out["oracle_plain_1m_first20k_k2"] = {"pairs": int(len(a)), "sha256": sha(a, b, d.astype(np.uint8))}
    path = os.path.join(ROOT, "tests", "golden", "oracle_results.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1, sort_keys=True)
    print(json.dumps(out, indent=1))


if __name__ == "__main__":
    main()
