"""The seeded input recipe: frame, lengths, residue law, mutant structure and
byte-for-byte determinism (golden hashes written by tests/golden/make_golden.py)."""
import hashlib
import json
import os

import numpy as np

import cdr3gen

HERE = os.path.dirname(os.path.abspath(__file__))
GOLD = json.load(open(os.path.join(HERE, "golden", "oracle_results.json")))


def sha(*arrays):
    h = hashlib.sha256()
    for a in arrays:
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()


def test_golden_hash_10k():
    assert sha(*cdr3gen.plain("plain_10k")) == GOLD["gen_plain_10k_sha256"]


def test_frame_and_lengths():
    c, o = cdr3gen.plain("plain_10k")
    L = np.diff(o)
    assert L.min() >= 8 and L.max() <= 24
    assert abs(L.mean() - 15.0) < 0.1
    assert np.all(c[o[:-1]] == cdr3gen.ALPHABET.index("C"))
    assert np.all(c[o[1:] - 1] == cdr3gen.ALPHABET.index("F"))
    assert c.max() < 20


def test_residue_law_is_zipf_over_a_fixed_permutation():
    p = cdr3gen.residue_probs()
    assert abs(p.sum() - 1) < 1e-12
    h20 = sum(1 / r for r in range(1, 21))
    assert np.allclose(np.sort(p)[::-1], [(1 / r) / h20 for r in range(1, 21)])
    c, o = cdr3gen.generate(99, 20000, fresh_frac=1.0)
    interior = np.concatenate([c[o[i] + 1:o[i + 1] - 1] for i in range(len(o) - 1)])
    freq = np.bincount(interior, minlength=20) / len(interior)
    assert np.max(np.abs(freq - p)) < 0.005


def test_mutants_are_near_earlier_sequences():
    import oracle
    c, o = cdr3gen.plain("plain_10k")
    s = cdr3gen.to_strings(c, o)
    # roughly 30 % of sequences sit within 2 edits of some earlier sequence
    a, b, d = oracle.self_search(c, o, 2)
    later = set(b.tolist())
    assert 0.25 < len(later) / len(s) < 0.35


def test_determinism_and_seed_dependence():
    a = cdr3gen.generate(5, 1000)
    b = cdr3gen.generate(5, 1000)
    c = cdr3gen.generate(6, 1000)
    assert sha(*a) == sha(*b) != sha(*c)


def test_query_sets_and_sizes():
    rc, ro = cdr3gen.generate(4, 5000)
    qc, qo = cdr3gen.generate_query(1000, 2000, rc, ro, ref_mut_frac=0.1)
    L = np.diff(qo)
    assert L.min() >= 8 and L.max() <= 24
    sizes = cdr3gen.loguniform_sizes(5, 512, 1000, 200000)
    assert sizes.min() >= 1000 and sizes.max() <= 200000
    assert abs(np.log(sizes).mean() - (np.log(1000) + np.log(200000)) / 2) < 0.25
    t = cdr3gen.poisson_arrivals(7, 4000, 50.0)
    assert np.all(np.diff(t) > 0) and abs(4000 / t[-1] - 50.0) < 5.0
