"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: numbers the
paper prints, textbook values, an independent construction (edit balls built
by applying edits, subsets from itertools), brute force over every pair, the
symmetric-deletion theorem, the bag-of-amino-acids bound, and the closed form
of the weighted score. A dropped DP term, a wrong index or a transposed
operand in the oracle fails at least one of them.
"""
import itertools
import json
import math
import os

import numpy as np
import pytest

import cdr3gen

HERE = os.path.dirname(os.path.abspath(__file__))
PINS = json.load(open(os.path.join(HERE, "golden", "paper_pins.json")))


def codes_of(s: str) -> bytes:
    return bytes(cdr3gen.ALPHABET.index(c) for c in s)


def csr(strings):
    """CSR (codes, offsets) from byte strings (any byte values)."""
    offs = np.zeros(len(strings) + 1, dtype=np.int64)
    offs[1:] = np.cumsum([len(s) for s in strings])
    return np.frombuffer(b"".join(strings), dtype=np.uint8).copy() if offs[-1] else np.zeros(0, np.uint8), offs


def triples(a, b, d):
    return list(zip(a.tolist(), b.tolist(), d.tolist()))


def all_strings(alphabet_size, max_len):
    out = []
    for L in range(max_len + 1):
        out.extend(bytes(t) for t in itertools.product(range(alphabet_size), repeat=L))
    return out


# ---------------------------------------------------------------- deletion variants

def test_deletion_variant_count_paper(oracle_lib):
    # Section II A: 56 deletion variants for a length-10 string at threshold 2
    s = codes_of("CASSLGQAYF")
    assert len(oracle_lib.variants(s, 2)) == PINS["deletion_variants_len10_k2"]["value"]


@pytest.mark.parametrize("L", [0, 1, 2, 5, 9, 15, 24])
@pytest.mark.parametrize("k", [0, 1, 2, 3])
def test_deletion_variants_are_all_subsequences(oracle_lib, L, k):
    # independent construction: keep every position subset of size >= L - k
    rng = np.random.default_rng(L * 10 + k)
    s = bytes(rng.integers(0, 20, size=L).tolist())
    got = oracle_lib.variants(s, k)
    want = []
    for m in range(0, min(k, L) + 1):
        for dele in itertools.combinations(range(L), m):
            want.append(bytes(s[x] for x in range(L) if x not in dele))
    assert got == want
    assert len(got) == sum(math.comb(L, m) for m in range(min(k, L) + 1))


# ---------------------------------------------------------------- Levenshtein DP

@pytest.mark.parametrize("a,b,d", [
    (b"kitten", b"sitting", 3), (b"flaw", b"lawn", 2), (b"", b"abc", 3), (b"abc", b"", 3),
    (b"", b"", 0), (b"abc", b"abc", 0), (b"intention", b"execution", 5),
    (b"saturday", b"sunday", 3), (b"ab", b"ba", 2), (b"abcdef", b"azced", 3),
])
def test_lev_textbook_values(oracle_lib, a, b, d):
    assert oracle_lib.lev(a, b) == d


def _edits(t, alphabet):
    out = set()
    L = len(t)
    for p in range(L):
        out.add(t[:p] + t[p + 1:])
        for c in alphabet:
            if c != t[p]:
                out.add(t[:p] + (c,) + t[p + 1:])
    for p in range(L + 1):
        for c in alphabet:
            out.add(t[:p] + (c,) + t[p:])
    return out


def test_lev_ball_paper_count(oracle_lib):
    # Section II A: 79,746 strings within distance 2 of a length-10 string.
    # Build the ball by applying edits (no DP), then require the DP to give
    # exactly the breadth-first edit count for every member.
    alphabet = tuple(range(20))
    s = tuple(range(3, 13))  # ten distinct residues
    r1 = _edits(s, alphabet) | {s}
    r2 = set(r1)
    for t in r1:
        r2 |= _edits(t, alphabet)
    assert len(r1) == 411
    assert len(r2) == PINS["levenshtein_ball_len10_r2"]["value"]
    members = sorted(r2)
    want = np.array([0 if t == s else (1 if t in r1 else 2) for t in members])
    c, o = csr([bytes(t) for t in members])
    got = oracle_lib.lev_one_to_many(bytes(s), c, o)
    assert np.array_equal(got, want)
    # a sample of the distance-3 shell: one more edit from the radius-2 ball
    rng = np.random.default_rng(0)
    shell = set()
    for idx in rng.choice(len(members), 300, replace=False):
        for t in _edits(members[idx], alphabet):
            if t not in r2:
                shell.add(t)
    shell = sorted(shell)[:5000]
    c, o = csr([bytes(t) for t in shell])
    assert np.all(oracle_lib.lev_one_to_many(bytes(s), c, o) == 3)


def test_lev_metric_properties(oracle_lib):
    rng = np.random.default_rng(1)
    for _ in range(400):
        la, lb, lc = rng.integers(0, 12, size=3)
        a, b, c = (bytes(rng.integers(0, 4, size=n).tolist()) for n in (la, lb, lc))
        dab, dba = oracle_lib.lev(a, b), oracle_lib.lev(b, a)
        assert dab == dba
        assert abs(la - lb) <= dab <= max(la, lb)
        assert oracle_lib.lev(a, a) == 0
        assert (dab == 0) == (a == b)
        if la == lb:
            assert dab <= sum(x != y for x, y in zip(a, b))
        assert oracle_lib.lev(a, c) <= dab + oracle_lib.lev(b, c)


# ---------------------------------------------------------------- SymDel search

def _exhaustive_set():
    strings = all_strings(3, 6)  # 1093 strings, lengths 0..6
    assert len(strings) == 1093
    return strings, csr(strings)


@pytest.mark.parametrize("k", [0, 1, 2, 3])
def test_symdel_equals_brute_force_exhaustive(oracle_lib, k):
    _, (c, o) = _exhaustive_set()
    got = triples(*oracle_lib.self_search(c, o, k))
    want = triples(*oracle_lib.brute_self(c, o, k))
    assert got == want
    assert (len(got) > 0) == (k > 0)  # the set has no duplicate strings


def test_brute_force_is_the_definition_tiny(oracle_lib):
    # pure-Python pair loop with an independent recursive distance
    from functools import lru_cache

    def rec(a, b):
        @lru_cache(None)
        def f(x, y):
            if x == 0:
                return y
            if y == 0:
                return x
            return min(f(x - 1, y) + 1, f(x, y - 1) + 1, f(x - 1, y - 1) + (a[x - 1] != b[y - 1]))
        return f(len(a), len(b))

    rng = np.random.default_rng(3)
    strings = [bytes(rng.integers(0, 3, size=rng.integers(0, 7)).tolist()) for _ in range(60)]
    c, o = csr(strings)
    for k in (1, 2):
        want = [(i, j, rec(strings[i], strings[j])) for i in range(60) for j in range(i + 1, 60)]
        want = [t for t in want if t[2] <= k]
        assert triples(*oracle_lib.self_search(c, o, k)) == want
        assert triples(*oracle_lib.brute_self(c, o, k)) == want


@pytest.mark.parametrize("k", [1, 2, 3])
def test_symmetric_deletion_theorem(oracle_lib, k):
    # Section II A / Fig. 1A-B: strings within k edits share a <=k-deletion
    # variant, so the candidate set contains every true pair.
    _, (c, o) = _exhaustive_set()
    ca, cb, raw = oracle_lib.self_candidates(c, o, k)
    cand = set(zip(ca.tolist(), cb.tolist()))
    a, b, _ = oracle_lib.brute_self(c, o, k)
    truth = set(zip(a.tolist(), b.tolist()))
    assert truth <= cand
    assert raw >= len(cand)


def test_duplicates_and_false_positives_fig1(oracle_lib):
    # Fig. 1C: one pair can match through several variants; Fig. 1D: a shared
    # variant does not imply distance <= k ("AC" and "CA" share "A" and "C").
    c, o = csr([codes_of("AC"), codes_of("CA")])
    ca, cb, raw = oracle_lib.self_candidates(c, o, 1)
    assert list(zip(ca, cb)) == [(0, 1)] and raw == 2
    a, _, _ = oracle_lib.self_search(c, o, 1)
    assert len(a) == 0
    assert oracle_lib.lev(codes_of("AC"), codes_of("CA")) == 2


def test_empty_variant_needed_for_short_strings(oracle_lib):
    # a length-1 and a length-2 string are within 2 edits and only share the
    # empty variant when every residue differs
    c, o = csr([codes_of("A"), codes_of("CD")])
    a, b, d = oracle_lib.self_search(c, o, 2)
    assert triples(a, b, d) == [(0, 1, 2)]


def test_duplicate_inputs_give_distance_zero(oracle_lib):
    c, o = csr([codes_of("CASSF"), codes_of("CASSF"), codes_of("CASTF")])
    assert triples(*oracle_lib.self_search(c, o, 1)) == [(0, 1, 0), (0, 2, 1), (1, 2, 1)]


def test_bag_of_amino_acids_bound(oracle_lib):
    # Appendix B theorem: ||bag(x) - bag(y)||^2 <= 2 d^2 for every output pair
    c, o = cdr3gen.plain("plain_10k")
    a, b, d = oracle_lib.self_search(c, o, 2)
    bags = np.zeros((len(o) - 1, 20), dtype=np.int64)
    seq_id = np.repeat(np.arange(len(o) - 1), np.diff(o))
    np.add.at(bags, (seq_id, c.astype(np.int64)), 1)
    diff = bags[a] - bags[b]
    assert np.all((diff * diff).sum(1) <= PINS["bag_bound_factor_sq"]["value"] * d.astype(np.int64) ** 2)


@pytest.mark.slow
def test_symdel_equals_brute_force_10k_config(oracle_lib):
    c, o = cdr3gen.plain("plain_10k")
    got = triples(*oracle_lib.self_search(c, o, 1))
    want = triples(*oracle_lib.brute_self(c, o, 1))
    assert got == want and len(got) > 1000


def test_symdel_equals_brute_force_generator_k2(oracle_lib):
    c, o = cdr3gen.subset(*cdr3gen.plain("plain_10k"), 2500)
    got = triples(*oracle_lib.self_search(c, o, 2))
    assert got == triples(*oracle_lib.brute_self(c, o, 2))
    assert {t[2] for t in got} == {0, 1, 2}


def test_symdel_equals_brute_force_generator_k3(oracle_lib):
    # Section III D's larger radius: SymDel at k = 3 against every pair
    c, o = cdr3gen.subset(*cdr3gen.plain("plain_10k"), 2500)
    got = triples(*oracle_lib.self_search(c, o, 3))
    assert got == triples(*oracle_lib.brute_self(c, o, 3))
    assert {t[2] for t in got} == {0, 1, 2, 3}


# ---------------------------------------------------------------- sharded mode

SHARDINGS = [(1, 1), (3, 2), (7, 3), (16, 4)]  # (shards, threads)


@pytest.mark.parametrize("k", [0, 1, 2, 3])
@pytest.mark.parametrize("shards,threads", SHARDINGS)
def test_sharded_equals_brute_force_exhaustive(oracle_lib, k, shards, threads):
    # every string of length <= 6 over 3 letters: the sharded run must give
    # brute force's triplets whatever the shard and thread counts
    _, (c, o) = _exhaustive_set()
    got = triples(*oracle_lib.self_search_sharded(c, o, k, shards=shards, threads=threads))
    assert got == triples(*oracle_lib.brute_self(c, o, k))


@pytest.mark.parametrize("shards,threads", SHARDINGS)
def test_sharded_equals_brute_force_generator_k2(oracle_lib, shards, threads):
    c, o = cdr3gen.subset(*cdr3gen.plain("plain_10k"), 2500)
    got = triples(*oracle_lib.self_search_sharded(c, o, 2, shards=shards, threads=threads))
    assert got == triples(*oracle_lib.brute_self(c, o, 2))


@pytest.mark.parametrize("k", [0, 1, 2])
def test_sharded_equals_plain_10k_config(oracle_lib, k):
    c, o = cdr3gen.plain("plain_10k")
    want = oracle_lib.self_search(c, o, k)
    for shards, threads in ((5, 4), (0, 0)):
        got = oracle_lib.self_search_sharded(c, o, k, shards=shards, threads=threads)
        assert all(np.array_equal(x, y) for x, y in zip(got, want))


def test_sharded_edge_cases(oracle_lib):
    # empty input, one sequence, more shards than variants
    c, o = csr([])
    assert len(oracle_lib.self_search_sharded(c, o, 2, shards=4, threads=2)[0]) == 0
    c, o = csr([codes_of("CASSF")])
    assert len(oracle_lib.self_search_sharded(c, o, 2, shards=4, threads=2)[0]) == 0
    c, o = csr([codes_of("A"), codes_of("CD"), codes_of("A")])
    got = triples(*oracle_lib.self_search_sharded(c, o, 2, shards=64, threads=8))
    assert got == [(0, 1, 2), (0, 2, 0), (1, 2, 2)]


@pytest.mark.parametrize("k", [0, 1, 2])
def test_query_equals_brute_force(oracle_lib, k):
    rc, ro = cdr3gen.generate(11, 1500)
    qc, qo = cdr3gen.generate_query(12, 700, rc, ro, ref_mut_frac=0.3)
    got = triples(*oracle_lib.query_search((rc, ro), (qc, qo), k))
    want = triples(*oracle_lib.brute_query((rc, ro), (qc, qo), k))
    assert got == want and len(got) > 0


# ---------------------------------------------------------------- Hamming mode

@pytest.mark.parametrize("a,b,d", [
    (b"karolin", b"kathrin", 3), (b"karolin", b"kerstin", 3), (b"1011101", b"1001001", 2),
    (b"2173896", b"2233796", 3), (b"", b"", 0), (b"abc", b"abc", 0), (b"abc", b"ab", -1),
    (b"a", b"", -1),
])
def test_hamming_textbook_values(oracle_lib, a, b, d):
    assert oracle_lib.hamming(a, b) == d


def test_hamming_brute_force_is_the_definition_tiny(oracle_lib):
    # pure-Python pair loop: equal lengths and at most k differing positions
    rng = np.random.default_rng(7)
    strings = [bytes(rng.integers(0, 3, size=rng.integers(0, 6)).tolist()) for _ in range(80)]
    c, o = csr(strings)
    for k in (0, 1, 2):
        want = []
        for i in range(80):
            for j in range(i + 1, 80):
                a, b = strings[i], strings[j]
                if len(a) == len(b):
                    d = sum(x != y for x, y in zip(a, b))
                    if d <= k:
                        want.append((i, j, d))
        assert triples(*oracle_lib.brute_self_hamming(c, o, k)) == want
        assert triples(*oracle_lib.self_search_hamming(c, o, k)) == want


@pytest.mark.parametrize("k", [0, 1, 2, 3])
def test_hamming_mode_equals_brute_force_exhaustive(oracle_lib, k):
    # Section III C: the SymDel candidates filtered by Hamming distance are
    # exactly the Hamming neighbours (Hamming <= k implies Levenshtein <= k)
    _, (c, o) = _exhaustive_set()
    got = triples(*oracle_lib.self_search_hamming(c, o, k))
    assert got == triples(*oracle_lib.brute_self_hamming(c, o, k))
    lev = set(triples(*oracle_lib.brute_self(c, o, k)))
    for i, j, d in got:  # every Hamming pair is a Levenshtein pair with Lev <= Hamming
        assert any((i, j, e) in lev for e in range(d + 1))


@pytest.mark.parametrize("k", [1, 2])
def test_hamming_mode_equals_brute_force_10k_config(oracle_lib, k):
    c, o = cdr3gen.plain("plain_10k")
    got = triples(*oracle_lib.self_search_hamming(c, o, k))
    assert got == triples(*oracle_lib.brute_self_hamming(c, o, k))
    assert len(got) > 500


@pytest.mark.parametrize("k", [1, 2])
def test_hamming_query_equals_brute_force(oracle_lib, k):
    rc, ro = cdr3gen.generate(11, 1500)
    qc, qo = cdr3gen.generate_query(12, 700, rc, ro, ref_mut_frac=0.3)
    got = triples(*oracle_lib.query_search_hamming((rc, ro), (qc, qo), k))
    assert got == triples(*oracle_lib.brute_query_hamming((rc, ro), (qc, qo), k))
    assert len(got) > 0


# ---------------------------------------------------------------- paired chains

def _token_aligned_distance(x: bytes, y: bytes, token: int = 255) -> int:
    """Edit distance of two joined records where the joining token can only
    be matched with the other token (deleting, inserting or substituting it
    is not allowed): a plain recursive DP, independent of the oracle."""
    from functools import lru_cache
    INF = 10 ** 6

    @lru_cache(None)
    def f(i, j):
        if i == 0 and j == 0:
            return 0
        best = INF
        if i > 0 and x[i - 1] != token:
            best = min(best, f(i - 1, j) + 1)
        if j > 0 and y[j - 1] != token:
            best = min(best, f(i, j - 1) + 1)
        if i > 0 and j > 0:
            a, b = x[i - 1], y[j - 1]
            if a == b:
                best = min(best, f(i - 1, j - 1))
            elif a != token and b != token:
                best = min(best, f(i - 1, j - 1) + 1)
        return best
    return f(len(x), len(y))


def test_paired_distance_is_token_aligned_edit_distance(oracle_lib):
    # the distance the paired mode reports, Lev(a) + Lev(b), is the edit
    # distance of the joined strings when the token must stay aligned
    rng = np.random.default_rng(11)
    for _ in range(400):
        a1, b1, a2, b2 = (bytes(rng.integers(0, 3, size=rng.integers(0, 5)).tolist()) for _ in range(4))
        want = _token_aligned_distance(a1 + b"\xff" + b1, a2 + b"\xff" + b2)
        assert oracle_lib.lev(a1, a2) + oracle_lib.lev(b1, b2) == want


@pytest.mark.parametrize("la,lb", [(0, 0), (1, 0), (3, 2), (10, 12), (15, 15), (24, 24)])
@pytest.mark.parametrize("k", [0, 1, 2, 3])
def test_paired_variant_count(oracle_lib, la, lb, k):
    a = bytes(range(la)) if la <= 20 else bytes(x % 20 for x in range(la))
    b = bytes(range(lb)) if lb <= 20 else bytes(x % 20 for x in range(lb))
    want = sum(math.comb(la, m1) * math.comb(lb, m2)
               for m1 in range(k + 1) for m2 in range(k + 1 - m1))
    assert oracle_lib.paired_variant_count(a, b, k) == want


def _paired_exhaustive():
    chains = [bytes(t) for L in range(1, 4) for t in itertools.product(range(2), repeat=L)]
    recs = [(x, y) for x in chains for y in chains]
    return csr([r[0] for r in recs]), csr([r[1] for r in recs])


@pytest.mark.parametrize("k", [0, 1, 2, 3])
def test_paired_equals_brute_force_exhaustive(oracle_lib, k):
    a, b = _paired_exhaustive()
    got = triples(*oracle_lib.paired_self_search(a, b, k))
    assert got == triples(*oracle_lib.brute_paired(a, b, k))
    assert (len(got) > 0) == (k > 0)


def paired_records(seed, n, fresh=500):
    """Records (a, b): the first `fresh` from the generator, the others a
    copy of an earlier record with a substitution in each chain, each with
    probability one half, so near pairs in both chains occur."""
    rng = np.random.default_rng(seed)
    ac, ao = cdr3gen.generate(seed, fresh)
    bc, bo = cdr3gen.generate(seed + 1, fresh)
    A = [ac[ao[x]:ao[x + 1]].tobytes() for x in range(fresh)]
    B = [bc[bo[x]:bo[x + 1]].tobytes() for x in range(fresh)]
    for i in range(fresh, n):
        u = int(rng.integers(i))
        x, y = bytearray(A[u]), bytearray(B[u])
        for z in (x, y):
            if rng.random() < 0.5:
                z[int(rng.integers(len(z)))] = int(rng.integers(20))
        A.append(bytes(x))
        B.append(bytes(y))
    return csr(A), csr(B)


@pytest.mark.parametrize("k", [1, 2, 3])
def test_paired_equals_brute_force_generator(oracle_lib, k):
    a, b = paired_records(61, 1500)
    got = triples(*oracle_lib.paired_self_search(a, b, k))
    assert got == triples(*oracle_lib.brute_paired(a, b, k))
    assert len(got) > 100


# ---------------------------------------------------------------- weighted score

def _closed_form_weighted(a: bytes, b: bytes, subst, indel=8, max_score=8):
    """Score if <= max_score else None, derived without any DP: with
    substitution costs in {3, 4} and indel cost 8, a score <= 8 needs equal
    lengths and at most two substitutions (the score is their cost sum), or
    lengths one apart with the shorter a one-deletion of the longer (score 8)."""
    if len(a) == len(b):
        mism = [(x, y) for x, y in zip(a, b) if x != y]
        s = sum(int(subst[x][y]) for x, y in mism)
        return s if s <= max_score else None
    if abs(len(a) - len(b)) == 1:
        lo, hi = (a, b) if len(a) < len(b) else (b, a)
        if any(hi[:p] + hi[p + 1:] == lo for p in range(len(hi))):
            return indel
    return None


def test_weighted_closed_form(oracle_lib):
    subst = cdr3gen.cost_matrix()
    assert np.array_equal(subst, subst.T) and np.all(np.diag(subst) == 0)
    off = subst[~np.eye(20, dtype=bool)]
    assert set(off.tolist()) == {3, 4}
    rng = np.random.default_rng(5)
    base = [bytes(rng.integers(0, 20, size=rng.integers(6, 12)).tolist()) for _ in range(40)]
    pool = []
    for s in base:  # near neighbours so that small scores occur often
        pool.append(s)
        t = bytearray(s)
        t[rng.integers(len(t))] = int(rng.integers(20))
        pool.append(bytes(t))
        p = int(rng.integers(len(s)))
        pool.append(s[:p] + s[p + 1:])
    for x in pool:
        for y in pool:
            w = oracle_lib.weighted(x, y, subst, 8)
            cf = _closed_form_weighted(x, y, subst)
            assert (w if w <= 8 else None) == cf
            if cf is not None:
                assert oracle_lib.lev(x, y) <= 2  # the k=2 lookup is an exact prefilter


def test_weighted_query_equals_brute_force(oracle_lib):
    subst = cdr3gen.cost_matrix()
    rc, ro = cdr3gen.generate(21, 1200)
    qc, qo = cdr3gen.generate_query(22, 600, rc, ro, ref_mut_frac=0.4)
    got = triples(*oracle_lib.query_weighted((rc, ro), (qc, qo), subst, 8, 8))
    want = triples(*oracle_lib.brute_weighted((rc, ro), (qc, qo), subst, 8, 8))
    assert got == want and len(got) > 0
    qs = cdr3gen.to_strings(qc, qo)
    rs = cdr3gen.to_strings(rc, ro)
    for q, r, s in got[:300]:
        assert _closed_form_weighted(codes_of(qs[q]), codes_of(rs[r]), subst) == s
