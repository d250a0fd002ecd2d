"""Hamming mode (paper Section III C: the method's candidates with the final
filter changed to Hamming distance) against the oracle's Hamming mode,
element by element: the 10K workload at k = 0, 1, 2 under the grouping and
pair-sort configurations, the exhaustive 3-letter set, a 20K prefix of the
1M workload, edge cases, the query path and the context option."""
import itertools

import numpy as np
import pytest

import cdr3gen

pytestmark = pytest.mark.gpu

CONFIGS = {
    "auto": {},
    "fullkey": {"path": 1},
    "counted_pairs": {"pair_sort": 2},
    "hashed_b20": {"path": 2, "bits": 20},
}


def log(msg):
    print(msg, flush=True)


def make_ctx(cfg):
    import torch
    from paper_2403_09010_amd import Context
    from paper_2403_09010_amd.symdel import OPT_GROUP_BITS, OPT_PAIR_SORT, OPT_PATH
    assert torch.cuda.is_available()
    c = Context(0)
    c.set_option(OPT_PATH, cfg.get("path", 0))
    c.set_option(OPT_GROUP_BITS, cfg.get("bits", 0))
    c.set_option(OPT_PAIR_SORT, cfg.get("pair_sort", 0))
    return c


@pytest.fixture(scope="module", params=sorted(CONFIGS))
def cctx(request):
    c = make_ctx(CONFIGS[request.param])
    c.name = request.param
    yield c
    c.close()


def to_dev(codes, offsets):
    import torch
    return (torch.from_numpy(np.ascontiguousarray(codes)).cuda(),
            torch.from_numpy(np.ascontiguousarray(offsets)).cuda())


def triples(r):
    i, j, d = r.numpy()
    return i.astype(np.uint32), j.astype(np.uint32), d.astype(np.int32)


def assert_same(got, want):
    assert len(got[0]) == len(want[0]), (len(got[0]), len(want[0]))
    for g, w in zip(got, want):
        assert np.array_equal(g, w.astype(g.dtype))


def csr(strings):
    offs = np.zeros(len(strings) + 1, dtype=np.int64)
    offs[1:] = np.cumsum([len(s) for s in strings])
    return np.frombuffer(b"".join(strings), dtype=np.uint8).copy(), offs


@pytest.mark.parametrize("k", [0, 1, 2])
def test_hamming_10k(cctx, k):
    import oracle
    c, o = cdr3gen.plain("plain_10k")
    log(f"self_search_hamming plain_10k k={k} config={cctx.name}")
    got = triples(cctx.self_search(*to_dev(c, o), k, hamming=True))
    want = oracle.self_search_hamming(c, o, k)
    assert_same(got, want)
    if k:
        assert len(want[0]) > 100


@pytest.mark.parametrize("k", [0, 1, 2])
def test_hamming_exhaustive_small_alphabet(cctx, k):
    import oracle
    strings = [bytes(t) for L in range(1, 7) for t in itertools.product(range(3), repeat=L)]
    c, o = csr(strings)
    log(f"self_search_hamming exhaustive 3-letter strings k={k} config={cctx.name}")
    assert_same(triples(cctx.self_search(*to_dev(c, o), k, hamming=True)),
                oracle.self_search_hamming(c, o, k))


def test_hamming_1m_prefix_20k():
    import oracle
    c, o = cdr3gen.subset(*cdr3gen.plain("plain_1m"), 20000)
    log("self_search_hamming first 20000 of plain_1m, k=2")
    ctx = make_ctx({})
    try:
        got = triples(ctx.self_search(*to_dev(c, o), 2, hamming=True))
    finally:
        ctx.close()
    assert_same(got, oracle.self_search_hamming(c, o, 2))


def test_hamming_edge_cases():
    import oracle
    ctx = make_ctx({})
    try:
        # lengths 1 and 24, copies, different lengths that are Levenshtein
        # neighbours but have no Hamming distance
        strings = [bytes([0]), bytes([5]), bytes([0, 1]), bytes([0]), bytes(range(20)) + bytes([1, 2, 3, 4]),
                   bytes(range(20)) + bytes([1, 2, 3, 5]), bytes(range(20)) + bytes([1, 2, 3]),
                   bytes([7, 8, 9]), bytes([7, 9, 8])]
        c, o = csr(strings)
        for k in (0, 1, 2):
            got = triples(ctx.self_search(c, o, k, hamming=True))
            assert_same(got, oracle.self_search_hamming(c, o, k))
        # (0, 2) are within Levenshtein 1 but never a Hamming pair
        got = triples(ctx.self_search(c, o, 2, hamming=True))
        assert (0, 2) not in set(zip(got[0].tolist(), got[1].tolist()))
    finally:
        ctx.close()


@pytest.mark.parametrize("k", [1, 2])
def test_hamming_query(k):
    import oracle
    ref = cdr3gen.generate(21, 6000)
    qry = cdr3gen.generate_query(22, 1500, *ref, ref_mut_frac=0.3)
    ctx = make_ctx({})
    try:
        idx = ctx.build_index(*to_dev(*ref), 2)
        log(f"query_hamming 1500 queries vs 6000 references, k={k}")
        got = triples(ctx.query(idx, *to_dev(*qry), k, hamming=True))
        want = oracle.query_search_hamming(ref, qry, k)
        assert_same(got, want)
        assert len(want[0]) > 0
        # the Levenshtein query on the same context is unchanged afterwards
        assert_same(triples(ctx.query(idx, *to_dev(*qry), k)), oracle.query_search(ref, qry, k))
        idx.free()
    finally:
        ctx.close()


def test_metric_option_equals_entry_point():
    from paper_2403_09010_amd.symdel import METRIC_HAMMING, METRIC_LEVENSHTEIN, OPT_METRIC
    c, o = cdr3gen.subset(*cdr3gen.plain("plain_10k"), 5000)
    ctx = make_ctx({})
    try:
        a = triples(ctx.self_search(*to_dev(c, o), 2, hamming=True))
        ctx.set_option(OPT_METRIC, METRIC_HAMMING)
        b = triples(ctx.self_search(*to_dev(c, o), 2))
        assert_same(b, a)
        ctx.set_option(OPT_METRIC, METRIC_LEVENSHTEIN)
        lev = triples(ctx.self_search(*to_dev(c, o), 2))
        assert len(lev[0]) > len(a[0])
    finally:
        ctx.close()
