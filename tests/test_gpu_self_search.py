"""Parity of the HIP self-search path with the CPU oracle (bit-exact: the
output is integer triplets). Small workloads are compared element by
element under every grouping and pair-sort configuration (so the branches
the full-size runs take are reached at small size too); the full 1M k=2 and
10M outputs are compared with the oracle's stored pair counts and hashes
(tests/golden, written by the oracle alone), plus sampled distances,
sampled completeness and properties that hold at any size."""
import hashlib
import json
import os

import numpy as np
import pytest

import cdr3gen

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))
GOLD = json.load(open(os.path.join(HERE, "golden", "oracle_results.json")))


def log(msg):
    print(msg, flush=True)


# grouping configurations: the automatic (hashed) path, the full-key sort
# path, and hashed runs with a small LDS capacity that send some or all hash
# segments through the oversized-segment fallback; with 18 or 20 hash bits
# the grouping sort takes three LSD passes (20 bits: digits at bits 44, 52
# and 60, the layout of the 10M workload); the automatic pair sort buckets
# the candidates by i and sorts each bucket in LDS, pair_sort forces the
# global counted passes (the branch above 2^22 sequences) or one-sweep passes
CONFIGS = {
    "auto": {},
    "fullkey": {"path": 1},
    "hashed_4096": {"path": 2, "cap": 4096},
    "hashed_2048_b18": {"path": 2, "cap": 2048, "bits": 18},
    "hashed_1024": {"path": 2, "cap": 1024},
    "hashed_cap256": {"path": 2, "cap": 256},
    "hashed_fallback": {"path": 2, "cap": 256, "bits": 4},
    "counted_pairs": {"pair_sort": 2},
    "hashed_b20_counted_pairs": {"path": 2, "bits": 20, "pair_sort": 2},
    "fullkey_counted_pairs": {"path": 1, "pair_sort": 2},
    "onesweep_pairs": {"pair_sort": 1},
}


def make_ctx(cfg):
    import torch
    from paper_2403_09010_amd import Context
    from paper_2403_09010_amd.symdel import (OPT_GROUP_BITS, OPT_GROUP_CAP, OPT_PAIR_SORT,
                                             OPT_PATH)
    assert torch.cuda.is_available()
    c = Context(0)
    c.set_option(OPT_PATH, cfg.get("path", 0))
    c.set_option(OPT_GROUP_CAP, cfg.get("cap", 0))
    c.set_option(OPT_GROUP_BITS, cfg.get("bits", 0))
    c.set_option(OPT_PAIR_SORT, cfg.get("pair_sort", 0))
    return c


@pytest.fixture(scope="module")
def ctx():
    c = make_ctx({})
    yield c
    c.close()


@pytest.fixture(scope="module", params=sorted(CONFIGS))
def cctx(request):
    c = make_ctx(CONFIGS[request.param])
    c.name = request.param
    c.cfg = CONFIGS[request.param]
    yield c
    c.close()


def to_dev(codes, offsets):
    import torch
    return (torch.from_numpy(np.ascontiguousarray(codes)).cuda(),
            torch.from_numpy(np.ascontiguousarray(offsets)).cuda())


def gpu_triples(ctx, codes, offsets, k, device=True):
    if device:
        r = ctx.self_search(*to_dev(codes, offsets), k)
    else:
        r = ctx.self_search(codes, offsets, k)
    i, j, d = r.numpy()
    return i.astype(np.uint32), j.astype(np.uint32), d.astype(np.int32)


def oracle_triples(codes, offsets, k):
    import oracle
    a, b, d = oracle.self_search(codes, offsets, k)
    return a, b, d


def assert_same(got, want):
    gi, gj, gd = got
    wi, wj, wd = want
    assert len(gi) == len(wi), (len(gi), len(wi))
    assert np.array_equal(gi, wi)
    assert np.array_equal(gj, wj)
    assert np.array_equal(gd, wd)


def csr(strings):
    offs = np.zeros(len(strings) + 1, dtype=np.int64)
    offs[1:] = np.cumsum([len(s) for s in strings])
    return np.frombuffer(b"".join(strings), dtype=np.uint8).copy(), offs


def sha(*arrays):
    h = hashlib.sha256()
    for a in arrays:
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()


# ---------------------------------------------------------------- distances

def test_pair_distance_exhaustive_small_alphabet(ctx):
    import itertools
    import torch
    import oracle
    strings = [bytes(t) for L in range(1, 7) for t in itertools.product(range(3), repeat=L)]
    c, o = csr(strings)
    rng = np.random.default_rng(0)
    ia = rng.integers(0, len(strings), 200000).astype(np.int32)
    ib = rng.integers(0, len(strings), 200000).astype(np.int32)
    log("pair_distance: 200000 pairs over 3-letter strings of length 1..6")
    d = ctx.pair_distance(to_dev(c, o), to_dev(c, o), torch.from_numpy(ia).cuda(),
                          torch.from_numpy(ib).cuda()).cpu().numpy()
    want = np.array([oracle.lev(strings[x], strings[y]) for x, y in zip(ia[:20000], ib[:20000])])
    assert np.array_equal(d[:20000], want)


def test_pair_distance_long_sequences(ctx):
    import torch
    import oracle
    c, o = cdr3gen.generate(77, 3000)
    rng = np.random.default_rng(1)
    ia = rng.integers(0, 3000, 20000).astype(np.int32)
    ib = rng.integers(0, 3000, 20000).astype(np.int32)
    log("pair_distance: 20000 random generator pairs")
    d = ctx.pair_distance(to_dev(c, o), to_dev(c, o), torch.from_numpy(ia).cuda(),
                          torch.from_numpy(ib).cuda()).cpu().numpy()
    seqs = [c[o[x]:o[x + 1]].tobytes() for x in range(3000)]
    want = np.array([oracle.lev(seqs[x], seqs[y]) for x, y in zip(ia, ib)])
    assert np.array_equal(d, want)


def test_pair_distance_rejects_bad_index(ctx):
    import torch
    from paper_2403_09010_amd import SymdelError
    c, o = cdr3gen.generate(3, 10)
    ia = torch.tensor([0, 10], dtype=torch.int32, device="cuda")
    ib = torch.tensor([1, 2], dtype=torch.int32, device="cuda")
    with pytest.raises(SymdelError) as e:
        ctx.pair_distance(to_dev(c, o), to_dev(c, o), ia, ib)
    assert e.value.code == -1


# ---------------------------------------------------------------- self search

@pytest.mark.parametrize("k", [0, 1, 2])
def test_plain_10k_matches_oracle(cctx, k):
    c, o = cdr3gen.plain("plain_10k")
    log(f"self_search plain_10k k={k} config={cctx.name}")
    got = gpu_triples(cctx, c, o, k)
    st = cctx.stats()
    assert_same(got, oracle_triples(c, o, k))
    # the bucketed pair sort is switched off (see
    # test_pair_bucket_over_the_workgroup_limit): every pair sort takes the
    # global passes
    assert st["n_pair_buckets"] == 0 and st["n_pair_fallbacks"] == 0
    g = GOLD[f"oracle_plain_10k_k{k}"]
    assert len(got[0]) == g["pairs"]
    assert sha(got[0], got[1], got[2].astype(np.uint8)) == g["sha256"]


def test_plain_1m_prefix_20k_k2_golden(cctx):
    c, o = cdr3gen.subset(*cdr3gen.plain("plain_1m"), 20000)
    log(f"self_search first 20000 of plain_1m, k=2 config={cctx.name}")
    got = gpu_triples(cctx, c, o, 2)
    g = GOLD["oracle_plain_1m_first20k_k2"]
    assert len(got[0]) == g["pairs"]
    assert sha(got[0], got[1], got[2].astype(np.uint8)) == g["sha256"]


@pytest.mark.parametrize("k", [0, 1, 2])
def test_exhaustive_small_alphabet(cctx, k):
    import itertools
    strings = [bytes(t) for L in range(1, 7) for t in itertools.product(range(3), repeat=L)]
    c, o = csr(strings)
    log(f"self_search exhaustive 3-letter strings, k={k} config={cctx.name}")
    assert_same(gpu_triples(cctx, c, o, k), oracle_triples(c, o, k))


def test_host_and_device_inputs_agree_and_repeat_bitwise(ctx):
    c, o = cdr3gen.generate(31, 30000)
    log("self_search host vs device inputs, 30000 sequences k=2")
    a = gpu_triples(ctx, c, o, 2, device=False)
    b = gpu_triples(ctx, c, o, 2, device=True)
    b2 = gpu_triples(ctx, c, o, 2, device=True)
    assert_same(a, b)
    assert_same(b, b2)


def test_edge_cases(cctx):
    ctx = cctx
    log(f"self_search edge cases config={cctx.name}")
    # empty input
    r = ctx.self_search(np.zeros(0, np.uint8), np.zeros(1, np.int64), 2)
    assert len(r) == 0
    # one sequence
    c, o = csr([bytes([1, 2, 3])])
    assert len(ctx.self_search(c, o, 2)) == 0
    # lengths 1 and 24, identical copies, tiny strings sharing only the empty variant
    strings = [bytes([0]), bytes([5, 6]), bytes([0]), bytes(range(20)) + bytes([1, 2, 3, 4]),
               bytes(range(20)) + bytes([1, 2, 3, 4]), bytes(range(20)) + bytes([1, 2, 3]),
               bytes([7]), bytes([8, 9])]
    c, o = csr(strings)
    for k in (0, 1, 2):
        assert_same(gpu_triples(ctx, c, o, k, device=False), oracle_triples(c, o, k))


def test_heavy_groups(cctx):
    # many copies of a few sequences: large groups of equal keys
    base, bo = cdr3gen.generate(41, 40)
    rng = np.random.default_rng(2)
    pick = rng.integers(0, 40, 3000)
    strings = [base[bo[x]:bo[x + 1]].tobytes() for x in pick]
    c, o = csr(strings)
    log(f"self_search heavy groups: 3000 sequences drawn from 40, config={cctx.name}")
    for k in (1, 2):
        assert_same(gpu_triples(cctx, c, o, k), oracle_triples(c, o, k))


def test_batches_of_shared_hashes(ctx):
    # 60 copies each of 40 sequences: every element of an LDS batch shares its
    # hash with others, so the grouping kernel's half-batch candidate table
    # overflows and lists each batch; the second pass, with a whole-batch
    # table, must group them all (nothing is left for the full-hash sort)
    base, bo = cdr3gen.generate(43, 40)
    rng = np.random.default_rng(5)
    pick = rng.permutation(np.repeat(np.arange(40), 60))
    strings = [base[bo[x]:bo[x + 1]].tobytes() for x in pick]
    c, o = csr(strings)
    for k in (1, 2):
        log(f"self_search 2400 sequences, 60 copies of each of 40, k={k}")
        assert_same(gpu_triples(ctx, c, o, k), oracle_triples(c, o, k))
        assert ctx.stats()["n_big_segments"] == 0


def test_group_larger_than_lds(ctx):
    # 4500 copies of one sequence: its variants form hash segments larger
    # than the 4096-element LDS capacity, so they take the full-key path
    import oracle
    x = cdr3gen.generate(51, 1)
    xs = x[0].tobytes()
    oc, oo = cdr3gen.generate(52, 300, fresh_frac=1.0)
    others = [oc[oo[t]:oo[t + 1]].tobytes() for t in range(300)]
    others = [t for t in others if t != xs]
    strings = [xs] * 4500 + others
    c, o = csr(strings)
    k = 1
    log("self_search 4500 identical sequences + 300 others, k=1")
    got = gpu_triples(ctx, c, o, k)
    st = ctx.stats()
    assert st["n_big_segments"] > 0
    want = []
    nx = 4500
    dx = [oracle.lev(xs, t) for t in others]
    for i in range(nx):
        for j in range(i + 1, nx):
            want.append((i, j, 0))
        for t, d in enumerate(dx):
            if d <= k:
                want.append((i, nx + t, d))
    oi, oj, od = oracle.self_search(*csr(others), k)
    want += [(nx + a, nx + b, d) for a, b, d in zip(oi.tolist(), oj.tolist(), od.tolist())]
    want.sort()
    w = np.array(want, dtype=np.int64)
    assert len(got[0]) == len(w)
    assert np.array_equal(got[0], w[:, 0]) and np.array_equal(got[1], w[:, 1])
    assert np.array_equal(got[2], w[:, 2])


@pytest.mark.skip(reason="the bucketed pair sort is switched off: its version with independent "
                         "buckets made the GPU take a memory fault on the first small self search "
                         "(10K sequences, k = 0), twice, cause not found yet")
def test_pair_bucket_over_the_workgroup_limit(ctx):
    # 1000 copies of one 24-residue sequence with no repeated residue at
    # k = 2: every pair of copies shares all 301 deletion variants, so the
    # first id's bucket holds 999 * 301 candidates, more than one workgroup
    # sorts (2^18): the whole array takes the global passes instead
    rng = np.random.default_rng(12)
    x = rng.permutation(20)
    s24 = bytes(np.concatenate([x, x[:4]]).astype(np.uint8))
    # no residue equals the next or the one after, so the 1 + 24 + 276
    # deletion sets give distinct strings
    assert all(s24[t] != s24[t + 1] for t in range(23)) and all(s24[t] != s24[t + 2] for t in range(22))
    c, o = csr([s24] * 1000)
    log("self_search 1000 copies of one 24-residue sequence, k=2")
    got = gpu_triples(ctx, c, o, 2)
    st = ctx.stats()
    assert st["n_pair_fallbacks"] == 1
    iu, ju = np.triu_indices(1000, 1)
    assert len(got[0]) == len(iu)
    assert np.array_equal(got[0], iu) and np.array_equal(got[1], ju)
    assert not got[2].any()


def test_budget_error_keeps_context_usable():
    from paper_2403_09010_amd import Context, SymdelError
    from paper_2403_09010_amd.symdel import OPT_STREAM
    log("self_search over a 4 MiB device budget (streaming off)")
    c, o = cdr3gen.plain("plain_10k")
    with Context(0, hbm_budget=4 << 20) as small:
        small.set_option(OPT_STREAM, 1)
        with pytest.raises(SymdelError) as e:
            small.self_search(*to_dev(c, o), 2)
        assert e.value.name == "SD_E_NOMEM"
        c2, o2 = cdr3gen.subset(c, o, 50)
        assert_same(gpu_triples(small, c2, o2, 1), oracle_triples(c2, o2, 1))


def test_paths_agree_at_full_size(ctx):
    c, o = cdr3gen.plain("plain_1m")
    log("self_search plain_1m k=2: hashed vs full-key path")
    a = gpu_triples(ctx, c, o, 2)
    full = make_ctx({"path": 1})
    try:
        b = gpu_triples(full, c, o, 2)
    finally:
        full.close()
    assert_same(a, b)


def test_errors(ctx):
    from paper_2403_09010_amd import SymdelError
    log("self_search error paths")
    c, o = csr([bytes([1, 2, 20])])
    with pytest.raises(SymdelError) as e:
        ctx.self_search(c, o, 1)
    assert e.value.name == "SD_E_ALPHABET"
    c, o = csr([bytes([1] * 25), bytes([1, 2])])
    with pytest.raises(SymdelError) as e:
        ctx.self_search(c, o, 1)
    assert e.value.name == "SD_E_LENGTH"
    c, o = csr([bytes([1, 2]), b""])
    with pytest.raises(SymdelError) as e:
        ctx.self_search(c, o, 1)
    assert e.value.name == "SD_E_LENGTH"
    c, o = csr([bytes([1, 2])])
    with pytest.raises(SymdelError) as e:
        ctx.self_search(c, o, 4)
    assert e.value.name == "SD_E_INVAL"
    # the context stays usable after errors
    c, o = cdr3gen.plain("plain_10k")
    assert_same(gpu_triples(ctx, c, o, 1), oracle_triples(c, o, 1))


# ---------------------------------------------------------------- full size

def assert_golden(got, name, n):
    """The whole output against the oracle's stored count and hash; on a
    mismatch, name the first id range whose chunk hash differs and print the
    GPU's first triplets there."""
    g = GOLD[name]
    i, j, d = got
    d8 = d.astype(np.uint8)
    if len(i) == g["pairs"] and sha(i, j, d8) == g["sha256"]:
        return
    chunks = len(g["chunk_sha256"])
    edges = np.searchsorted(i, [n * x // chunks for x in range(chunks + 1)])
    for x, (lo, hi) in enumerate(zip(edges[:-1], edges[1:])):
        if sha(i[lo:hi], j[lo:hi], d8[lo:hi]) != g["chunk_sha256"][x]:
            first = list(zip(i[lo:lo + 5].tolist(), j[lo:lo + 5].tolist(), d[lo:lo + 5].tolist()))
            pytest.fail(f"{name}: {len(i)} pairs against {g['pairs']}; first differing id range "
                        f"[{n * x // chunks}, {n * (x + 1) // chunks}) holds {hi - lo} GPU "
                        f"triplets, the first ones {first}")
    pytest.fail(f"{name}: {len(i)} pairs against {g['pairs']}, hash differs")


@pytest.mark.parametrize("cfg", ["auto", "counted_pairs", "onesweep_pairs", "fullkey"])
def test_plain_1m_k2_equals_oracle(cfg):
    """Every triplet of the headline workload equals the oracle's (count and
    hash of the whole output), through the automatic path (bucketed pair
    sort), the counted and one-sweep pair sorts and the full-key grouping
    path."""
    c, o = cdr3gen.plain("plain_1m")
    conf = {"auto": {}, "counted_pairs": {"pair_sort": 2}, "onesweep_pairs": {"pair_sort": 1},
            "fullkey": {"path": 1}}[cfg]
    log(f"self_search plain_1m k=2 config={cfg} against the oracle golden")
    ctx = make_ctx(conf)
    try:
        got = gpu_triples(ctx, c, o, 2)
    finally:
        ctx.close()
    assert_golden(got, "oracle_plain_1m_k2", len(o) - 1)


@pytest.mark.parametrize("k", [1, 2])
def test_plain_10m_equals_oracle(ctx, k):
    """The 10M workload (40% cluster members; three hash passes, counted
    pair sort) against the oracle's stored count and hash."""
    name = f"oracle_plain_10m_k{k}"
    if name not in GOLD:
        pytest.skip(f"{name} is not in tests/golden (make_golden.py --only {name})")
    c, o = cdr3gen.plain("plain_10m")
    log(f"self_search plain_10m k={k} against the oracle golden")
    got = gpu_triples(ctx, c, o, k)
    assert_golden(got, name, len(o) - 1)


def test_plain_1m_k2_sampled(ctx):
    import oracle
    c, o = cdr3gen.plain("plain_1m")
    n = len(o) - 1
    log("self_search plain_1m k=2 (full size)")
    i, j, d = gpu_triples(ctx, c, o, 2)
    assert len(i) > 300000
    # sorted, unique, i < j
    key = (i.astype(np.uint64) << np.uint64(32)) | j.astype(np.uint64)
    assert np.all(i < j) and np.all(np.diff(key.astype(np.int64)) > 0)
    assert d.min() >= 0 and d.max() <= 2
    # sampled outputs: exact distances
    rng = np.random.default_rng(5)
    seqs = lambda x: c[o[x]:o[x + 1]].tobytes()
    for t in rng.choice(len(i), 3000, replace=False):
        assert oracle.lev(seqs(i[t]), seqs(j[t])) == d[t]
    # sampled completeness: every neighbour of 40 random sequences is reported
    for x in rng.choice(n, 40, replace=False):
        dist = oracle.lev_one_to_many(seqs(x), c, o)
        truth = {(min(x, y), max(x, y), int(dist[y])) for y in np.nonzero(dist <= 2)[0] if y != x}
        mine = set()
        for sel in (np.nonzero(i == x)[0], np.nonzero(j == x)[0]):
            mine |= {(int(i[t]), int(j[t]), int(d[t])) for t in sel}
        assert mine == truth
    # bag-of-amino-acids bound (Appendix B) on every output pair
    bags = np.zeros((n, 20), dtype=np.int16)
    seq_id = np.repeat(np.arange(n), np.diff(o))
    np.add.at(bags, (seq_id, c.astype(np.int64)), 1)
    diff = (bags[i] - bags[j]).astype(np.int64)
    assert np.all((diff * diff).sum(1) <= 2 * d.astype(np.int64) ** 2)


@pytest.mark.parametrize("k,samples", [(1, 4), (2, 6)])
def test_plain_10m_sampled(ctx, k, samples):
    """10M sequences with 40% cluster members: properties of the whole output,
    exact distances of sampled pairs and every neighbour of sampled sequences."""
    import oracle
    c, o = cdr3gen.plain("plain_10m")
    n = len(o) - 1
    log(f"self_search plain_10m k={k} (full size)")
    i, j, d = gpu_triples(ctx, c, o, k)
    log(f"  {len(i)} pairs")
    assert len(i) > (1_000_000 if k == 2 else 500_000)
    key = (i.astype(np.uint64) << np.uint64(32)) | j.astype(np.uint64)
    assert np.all(i < j) and np.all(np.diff(key.astype(np.int64)) > 0)
    assert d.max() <= k
    rng = np.random.default_rng(10 + k)
    seqs = lambda x: c[o[x]:o[x + 1]].tobytes()
    for t in rng.choice(len(i), 2000, replace=False):
        assert oracle.lev(seqs(i[t]), seqs(j[t])) == d[t]
    # completeness: half the samples are reported sequences (they have
    # neighbours), half are uniform
    picks = list(rng.choice(i, samples // 2)) + list(rng.choice(n, samples - samples // 2))
    order = np.argsort(i, kind="stable")
    i_sorted = i[order]
    order_j = np.argsort(j, kind="stable")
    j_sorted = j[order_j]
    for x in picks:
        dist = oracle.lev_one_to_many(seqs(x), c, o)
        truth = {(min(x, y), max(x, y), int(dist[y])) for y in np.nonzero(dist <= k)[0] if y != x}
        a0, a1 = np.searchsorted(i_sorted, x), np.searchsorted(i_sorted, x, side="right")
        b0, b1 = np.searchsorted(j_sorted, x), np.searchsorted(j_sorted, x, side="right")
        sel = np.concatenate([order[a0:a1], order_j[b0:b1]])
        mine = {(int(i[t]), int(j[t]), int(d[t])) for t in sel}
        assert mine == truth, f"sequence {x}"
