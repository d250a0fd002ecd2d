"""The rule by which the hashed path generates each distinct deletion variant
of a sequence once (the GPU keeps only "canonical" deletion sets; their
count per sequence sizes the variant offsets).

Deleting a set D of at most two positions from s gives a string t; the
greedy leftmost embedding of t in s deletes a unique set D*(t). For |D| <= 2
the test D == D* is local (see variant_canonical in the device header):

  {p}       : p = L-1 or s[p] != s[p+1]
  {p1 < p2} : (p2 = L-1 or s[p2] != s[p2+1]) and
              (s[p1] != s[p1+1] if p2 > p1+1, else p2 = L-1 or s[p1] != s[p1+2])

and the number of canonical sets has the O(L) form used by the pack kernel.
These checks hold the rule against brute force: every distinct variant string
has exactly one canonical deletion set, and the count matches. The variant
set itself is the paper's (Section II A); the rule only drops repeats of the
same string, so the pairs found are unchanged.
"""
import itertools
import random

import pytest


def variants(s, k):
    """Every deletion set with at most k positions and the string it leaves."""
    L = len(s)
    out = [((), s)]
    for m in range(1, min(k, L) + 1):
        for D in itertools.combinations(range(L), m):
            out.append((D, "".join(c for i, c in enumerate(s) if i not in D)))
    return out


def greedy_deleted(s, t):
    """Positions of s left out by the greedy leftmost embedding of t."""
    j, dele = 0, []
    for i, c in enumerate(s):
        if j < len(t) and c == t[j]:
            j += 1
        else:
            dele.append(i)
    assert j == len(t)
    return tuple(dele)


def canonical(s, D):
    L = len(s)
    if len(D) == 0:
        return True
    if len(D) == 1:
        p = D[0]
        return p == L - 1 or s[p] != s[p + 1]
    p1, p2 = D
    b = p2 == L - 1 or s[p2] != s[p2 + 1]
    if p1 + 1 < p2:
        a = s[p1] != s[p1 + 1]
    else:
        a = p2 == L - 1 or s[p1] != s[p1 + 2]
    return a and b


def distinct_count(s, k):
    """The O(L) count of canonical sets (the pack kernel's form)."""
    L = len(s)
    c = 1
    if k >= 1:
        c += sum(1 for p in range(L) if p == L - 1 or s[p] != s[p + 1])
    if k >= 2:
        run = 0  # canonical first deletions p1 <= p2 - 2
        for p2 in range(1, L):
            if p2 >= 2 and s[p2 - 2] != s[p2 - 1]:
                run += 1
            if p2 == L - 1 or s[p2] != s[p2 + 1]:
                c += run
                if p2 == L - 1 or s[p2 - 1] != s[p2 + 1]:
                    c += 1
    return c


def masks(s):
    """n1 bit p: p = L-1 or s[p] != s[p+1]; n2 bit p: p = L-2 or s[p] != s[p+2]."""
    L = len(s)
    n1 = sum(1 << p for p in range(L) if p == L - 1 or s[p] != s[p + 1])
    n2 = sum(1 << p for p in range(L - 1) if p == L - 2 or s[p] != s[p + 2])
    return n1, n2


def distinct_count_masks(s, k):
    """The same count from the two masks, as the pack kernel computes it."""
    L = len(s)
    n1, n2 = masks(s)
    c = 1
    if k >= 1:
        c += bin(n1).count("1")
    if k >= 2:
        for p2 in range(1, L):
            if (n1 >> p2) & 1:
                c += bin(n1 & ((1 << (p2 - 1)) - 1)).count("1") + ((n2 >> (p2 - 1)) & 1)
    return c


def canonical_masks(s, D):
    """variant_canonical's test on the masks."""
    L = len(s)
    n1, n2 = masks(s)
    if len(D) == 0:
        return True
    if len(D) == 1:
        return bool((n1 >> D[0]) & 1)
    p1, p2 = D
    a = (n1 >> p1) if p1 + 1 < p2 else (n2 >> p1)
    return bool(a & (n1 >> p2) & 1)


def canonical_ext(s, D):
    """The generator's form with no case split: one deletion at p is the
    position pair (p, L), no deletion is (L, L + 1), and the masks gain bits
    L, L + 1 (n1) and L - 1, L (n2)."""
    L = len(s)
    n1, n2 = masks(s)
    n1x = n1 | (3 << L)
    n2x = n2 | (1 << L) | ((1 << (L - 1)) if L >= 1 else 0)
    if len(D) == 0:
        p1, p2 = L, L + 1
    elif len(D) == 1:
        p1, p2 = D[0], L
    else:
        p1, p2 = D
    sel = n1x if p2 > p1 + 1 else n2x
    return bool((sel >> p1) & (n1x >> p2) & 1)


def random_strings(n, seed):
    rng = random.Random(seed)
    for _ in range(n):
        L = rng.randint(1, 10)
        alphabet = "ACDEFGHIKLMNPQRSTVWY"[: rng.choice([1, 2, 3, 20])]
        yield "".join(rng.choice(alphabet) for _ in range(L))


@pytest.mark.parametrize("k", [0, 1, 2])
def test_one_canonical_set_per_distinct_string(k):
    for s in random_strings(3000, 11 + k):
        by_string = {}
        for D, t in variants(s, k):
            by_string.setdefault(t, []).append(D)
        for t, Ds in by_string.items():
            canon = [D for D in Ds if canonical(s, D)]
            assert len(canon) == 1, (s, t, Ds)
            # the canonical set is the greedy embedding's
            assert canon[0] == greedy_deleted(s, t), (s, t)


@pytest.mark.parametrize("k", [0, 1, 2])
def test_distinct_count_formula(k):
    for s in random_strings(3000, 23 + k):
        distinct = len({t for _, t in variants(s, k)})
        assert distinct_count(s, k) == distinct, s
        assert distinct_count_masks(s, k) == distinct, s


@pytest.mark.parametrize("k", [1, 2])
def test_mask_form_of_the_rule(k):
    for s in random_strings(2000, 37 + k):
        for D, _ in variants(s, k):
            assert canonical_masks(s, D) == canonical(s, D), (s, D)


def test_worked_cases():
    # a run of equal residues: deleting any one of "AAA" gives the same string
    assert distinct_count("AAA", 1) == 2          # "AAA", "AA"
    assert distinct_count("AAA", 2) == 3          # + "A"
    # the periodic case that a shift-left rule gets wrong: ABAB minus two
    # adjacent positions gives "AB" three ways and "BA" once
    assert sorted(t for D, t in variants("ABAB", 2) if len(D) == 2 and canonical("ABAB", D)) == \
        ["AA", "AB", "BA", "BB"]
    # no repeated residues: every deletion set is canonical
    s = "ACDEFGHIKL"
    assert distinct_count(s, 2) == 1 + 10 + 45


@pytest.mark.parametrize("k", [0, 1, 2])
def test_extended_mask_form_of_the_rule(k):
    for s in list(random_strings(2000, 41 + k)) + ["", "A", "AA", "AB", "AAA"]:
        for D, _ in variants(s, k):
            assert canonical_ext(s, D) == canonical(s, D), (s, D)


# ---------------------------------------------------------------- k = 3
#
# For any D the greedy test reads: every deleted position p whose next kept
# position q(p) exists must hold a different residue (s[p] != s[q(p)]). For
# |D| <= 3, q(p) is p + 1, p + 2 or p + 3, so three masks suffice: n1, n2 and
# n3 bit p = (p >= L - 3 or s[p] != s[p + 3]). The generator enumerates
# every set as a padded triple p1 < p2 < p3 (a pair is (p1, p2, L), one
# deletion (p1, L, L + 1), none (L, L + 1, L + 2)); positions >= L are not
# deletions.

def canonical_general(s, D):
    """The greedy rule for any deletion set."""
    L, Dset = len(s), set(D)
    for p in D:
        q = p + 1
        while q in Dset:
            q += 1
        if q < L and s[p] == s[q]:
            return False
    return True


def masks3(s):
    L = len(s)
    n1, n2 = masks(s)
    n3 = sum(1 << p for p in range(L) if p >= L - 3 or s[p] != s[p + 3])
    return n1, n2, n3


def padded(D, L):
    D = tuple(D) + tuple(range(L, L + 3 - len(D)))
    return D


def canonical_triple(s, D):
    """The generator's test on a padded triple and the extended masks (n2
    gains bits L - 1 and L, as in canonical_ext; n1 gains L and L + 1)."""
    L = len(s)
    n1, n2, n3 = masks3(s)
    n1x = n1 | (3 << L)
    n2x = n2 | (1 << L) | ((1 << (L - 1)) if L >= 1 else 0)
    p1, p2, p3 = padded(D, L)
    real2, real3 = p2 < L, p3 < L
    c3 = not real3 or (n1x >> p3) & 1
    c2 = not real2 or ((n2x if (real3 and p3 == p2 + 1) else n1x) >> p2) & 1
    if p1 >= L:
        c1 = 1
    elif p2 > p1 + 1:
        c1 = (n1x >> p1) & 1
    elif real2 and real3 and p3 == p2 + 1:
        c1 = (n3 >> p1) & 1
    else:
        c1 = (n2x >> p1) & 1
    return bool(c1 and c2 and c3)


def distinct_count3_masks(s):
    """Canonical sets of exactly three deletions in O(L^2) from the masks
    (the pack kernel's form): for each canonical (p2, p3), the first
    deletions p1 <= p2 - 2 need n1, and p1 = p2 - 1 needs n2 (p3 > p2 + 1)
    or n3 (p3 = p2 + 1)."""
    L = len(s)
    n1, n2, n3 = masks3(s)
    c = 0
    for p3 in range(2, L):
        if not (n1 >> p3) & 1:
            continue
        for p2 in range(1, p3):
            adj = p3 == p2 + 1
            if not ((n2 if adj else n1) >> p2) & 1:
                continue
            c += bin(n1 & ((1 << (p2 - 1)) - 1)).count("1") if p2 >= 1 else 0
            c += ((n3 if adj else n2) >> (p2 - 1)) & 1
    return c


@pytest.mark.parametrize("k", [0, 1, 2, 3])
def test_general_rule_one_set_per_distinct_string(k):
    for s in random_strings(1500, 51 + k):
        by_string = {}
        for D, t in variants(s, k):
            by_string.setdefault(t, []).append(D)
        for t, Ds in by_string.items():
            canon = [D for D in Ds if canonical_general(s, D)]
            assert canon == [greedy_deleted(s, t)], (s, t, Ds)
        if k <= 2:
            for D, _ in variants(s, k):
                assert canonical_general(s, D) == canonical(s, D), (s, D)


def test_padded_triple_form_of_the_rule():
    for s in list(random_strings(1500, 61)) + ["", "A", "AA", "AAA", "AAAA", "ABAB", "ABCABC"]:
        for D, _ in variants(s, 3):
            assert canonical_triple(s, D) == canonical_general(s, D), (s, D)


def test_distinct_count_k3():
    for s in list(random_strings(2000, 71)) + ["A", "AA", "AAA", "AAAA", "ABAB", "ABCABC"]:
        distinct3 = len({t for D, t in variants(s, 3) if len(D) == 3})
        assert distinct_count3_masks(s) == distinct3, s
        # strings with exactly three deletions never equal shorter-deletion ones
        assert distinct_count_masks(s, 2) + distinct3 == len({t for _, t in variants(s, 3)}), s
    assert distinct_count3_masks("ACDEFGHIKL") == 120
