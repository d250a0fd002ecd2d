"""Parity of the HIP query-versus-reference path (index build, single query,
batched query sets, weighted rescoring) with the CPU oracle, bit-exact."""
import numpy as np
import pytest

import cdr3gen

pytestmark = pytest.mark.gpu


def log(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_2403_09010_amd import Context
    assert torch.cuda.is_available()
    c = Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def ref():
    return cdr3gen.generate(11, 3000)


@pytest.fixture(scope="module")
def index2(ctx, ref):
    idx = ctx.build_index(*ref, 2)
    yield idx
    idx.free()


def to_dev(codes, offsets):
    import torch
    return (torch.from_numpy(np.ascontiguousarray(codes)).cuda(),
            torch.from_numpy(np.ascontiguousarray(offsets)).cuda())


def triples(r):
    i, j, d = r.numpy()
    return list(zip(i.astype(np.int64).tolist(), j.astype(np.int64).tolist(),
                    d.astype(np.int64).tolist()))


def oracle_query(ref, qry, k):
    import oracle
    a, b, d = oracle.query_search(ref, qry, k)
    return list(zip(a.tolist(), b.tolist(), d.tolist()))


def csr(strings):
    offs = np.zeros(len(strings) + 1, dtype=np.int64)
    offs[1:] = np.cumsum([len(s) for s in strings])
    return np.frombuffer(b"".join(strings), dtype=np.uint8).copy(), offs


@pytest.mark.parametrize("k", [0, 1, 2])
def test_query_matches_oracle(ctx, ref, index2, k):
    qry = cdr3gen.generate_query(12, 1500, *ref, ref_mut_frac=0.3)
    log(f"query 1500 vs 3000 reference, k={k}")
    got = triples(ctx.query(index2, *to_dev(*qry), k))
    want = oracle_query(ref, qry, k)
    assert got == want and (k == 0 or len(got) > 100)


def test_index_with_its_own_k(ctx, ref):
    qry = cdr3gen.generate_query(13, 800, *ref, ref_mut_frac=0.3)
    idx = ctx.build_index(*ref, 1)
    try:
        log("query against a k=1 index")
        assert triples(ctx.query(idx, *qry, 1)) == oracle_query(ref, qry, 1)
        info = idx.info()
        assert info["n_ref"] == 3000 and info["k"] == 1 and info["n_keys"] > 3000
        from paper_2403_09010_amd import SymdelError
        with pytest.raises(SymdelError) as e:
            ctx.query(idx, *qry, 2)
        assert e.value.name == "SD_E_INVAL"
    finally:
        idx.free()


def test_batch_equals_single_queries(ctx, ref, index2):
    from paper_2403_09010_amd.symdel import OPT_BATCH_TILE
    sizes = [700, 0, 1, 1200, 50, 900, 333]
    sets = [cdr3gen.generate_query(100 + x, n, *ref, ref_mut_frac=0.2) if n else
            (np.zeros(0, np.uint8), np.zeros(1, np.int64)) for x, n in enumerate(sizes)]
    for tile in (0, 1000):  # one tile, then several tiles
        ctx.set_option(OPT_BATCH_TILE, tile)
        log(f"query_batch of {len(sets)} sets, tile limit {tile}")
        outs = ctx.query_batch(index2, [to_dev(*s) for s in sets], 2)
        for s, o in zip(sets, outs):
            want = oracle_query(ref, s, 2) if len(s[1]) > 1 else []
            assert triples(o) == want
        outs_h = ctx.query_batch(index2, sets, 2, device_output=False)
        for o, oh in zip(outs, outs_h):
            assert triples(o) == triples(oh)
    ctx.set_option(OPT_BATCH_TILE, 0)


def test_weighted_matches_oracle(ctx, ref, index2):
    import oracle
    subst = cdr3gen.cost_matrix()
    qry = cdr3gen.generate_query(14, 1500, *ref, ref_mut_frac=0.4)
    log("weighted query 1500 vs 3000, costs {3,4}, indel 8, max 8")
    got = triples(ctx.query_weighted(index2, *to_dev(*qry), subst, 8, 8))
    a, b, d = oracle.query_weighted(ref, qry, subst, 8, 8)
    want = list(zip(a.tolist(), b.tolist(), d.tolist()))
    assert got == want and len(got) > 50
    # a looser threshold keeps more pairs, all within the Levenshtein prefilter
    got2 = triples(ctx.query_weighted(index2, *to_dev(*qry), subst, 8, 16))
    a, b, d = oracle.query_weighted(ref, qry, subst, 8, 16)
    assert got2 == list(zip(a.tolist(), b.tolist(), d.tolist()))


def test_index_segment_larger_than_lds(ctx):
    # 5000 copies of one reference sequence: its variants fill index segments
    # beyond the join kernel's LDS capacity, which then search global memory
    x = cdr3gen.generate(61, 1)
    xs = x[0].tobytes()
    others = cdr3gen.generate(62, 500, fresh_frac=1.0)
    ostr = [others[0][others[1][t]:others[1][t + 1]].tobytes() for t in range(500)]
    rstrings = [xs] * 5000 + ostr
    rc = csr(rstrings)
    q = cdr3gen.generate_query(63, 60, *csr([xs]), ref_mut_frac=1.0)
    qc = (np.concatenate([q[0], others[0][:others[1][40]]]),
          np.concatenate([q[1], q[1][-1] + others[1][1:41]]))
    log("query against a reference with 5000 identical sequences")
    idx = ctx.build_index(*rc, 1)
    try:
        got = triples(ctx.query(idx, *to_dev(*qc), 1))
    finally:
        idx.free()
    assert got == oracle_query(rc, qc, 1)
    assert len(got) > 5000


def test_query_errors_and_empty(ctx, ref, index2):
    from paper_2403_09010_amd import SymdelError
    log("query error paths")
    assert len(ctx.query(index2, np.zeros(0, np.uint8), np.zeros(1, np.int64), 2)) == 0
    c, o = csr([bytes([1, 2, 25])])
    with pytest.raises(SymdelError) as e:
        ctx.query(index2, c, o, 2)
    assert e.value.name == "SD_E_ALPHABET"
    qry = cdr3gen.generate_query(15, 200, *ref, ref_mut_frac=0.5)
    assert triples(ctx.query(index2, *qry, 2)) == oracle_query(ref, qry, 2)


def test_query_at_scale_sampled(ctx):
    import oracle
    rc, ro = cdr3gen.generate(4, 200000)
    qc, qo = cdr3gen.generate_query(1000, 20000, rc, ro, ref_mut_frac=0.1)
    log("query 20000 vs 200000 reference, k=2")
    idx = ctx.build_index(*to_dev(rc, ro), 2)
    try:
        i, j, d = ctx.query(idx, *to_dev(qc, qo), 2).numpy()
    finally:
        idx.free()
    key = (i.astype(np.int64) << 32) | j.astype(np.int64)
    assert np.all(np.diff(key) > 0)
    rng = np.random.default_rng(3)
    seq = lambda c, o, x: c[o[x]:o[x + 1]].tobytes()
    for t in rng.choice(len(i), min(2000, len(i)), replace=False):
        assert oracle.lev(seq(qc, qo, i[t]), seq(rc, ro, j[t])) == d[t]
    for x in rng.choice(20000, 15, replace=False):
        dist = oracle.lev_one_to_many(seq(qc, qo, x), rc, ro)
        truth = {(int(x), int(r), int(dist[r])) for r in np.nonzero(dist <= 2)[0]}
        sel = np.nonzero(i == x)[0]
        assert {(int(i[t]), int(j[t]), int(d[t])) for t in sel} == truth


def test_batch_of_24_sets_against_oracle(ctx, ref, index2):
    """24 query sets of log-uniform sizes (one empty, one larger than the
    tile limit) in one batched call: every set's result equals the oracle's
    query of that set alone, under the automatic tiling and under a tile
    limit that puts the sets into many tiles."""
    from paper_2403_09010_amd.symdel import OPT_BATCH_TILE
    sizes = [int(x) for x in cdr3gen.loguniform_sizes(77, 24, 20, 2500)]
    sizes[5] = 0
    sizes[11] = 3200  # larger than the 1500-sequence tile limit below
    sets = [cdr3gen.generate_query(300 + x, n, *ref, ref_mut_frac=0.25) if n else
            (np.zeros(0, np.uint8), np.zeros(1, np.int64)) for x, n in enumerate(sizes)]
    want = [oracle_query(ref, s, 2) if len(s[1]) > 1 else [] for s in sets]
    assert sum(len(w) for w in want) > 500
    for tile in (0, 1500):
        ctx.set_option(OPT_BATCH_TILE, tile)
        log(f"query_batch of 24 sets ({sum(sizes)} sequences), tile limit {tile}")
        outs = ctx.query_batch(index2, [to_dev(*s) for s in sets], 2)
        for x, (o, w) in enumerate(zip(outs, want)):
            assert triples(o) == w, f"set {x} (size {sizes[x]}) differs from the oracle"
    ctx.set_option(OPT_BATCH_TILE, 0)


@pytest.mark.parametrize("n", [1, 10, 300, 3000])
def test_small_queries_join_coarser_segments(ctx, n):
    """A query tile with few variants joins over coarser segments than the
    index's own (unions of index segments found in its sorted array); with
    SD_OPT_JOIN_ELEMS = 1 every tile keeps the index's own segments. Both
    equal the oracle for 1 to 3,000 queries against a 20,000-sequence
    index, plain and weighted."""
    import oracle
    from paper_2403_09010_amd.symdel import OPT_JOIN_ELEMS
    big = cdr3gen.generate(19, 20_000)
    qry = cdr3gen.generate_query(90 + n, n, *big, ref_mut_frac=0.5)
    subst = cdr3gen.cost_matrix(8, 3, 4)
    a, b, d = oracle.query_weighted(big, qry, subst, 8, 8)
    want_w = list(zip(a.tolist(), b.tolist(), d.tolist()))
    want = {k: oracle_query(big, qry, k) for k in (1, 2)}
    idx = ctx.build_index(*to_dev(*big), 2)
    try:
        for per in (0, 1):
            ctx.set_option(OPT_JOIN_ELEMS, per)
            log(f"{n} queries against 20K, join elements option {per}")
            for k in (1, 2):
                assert triples(ctx.query(idx, *qry, k)) == want[k], f"k={k}"
            assert triples(ctx.query_weighted(idx, *qry, subst, 8, 8)) == want_w
    finally:
        ctx.set_option(OPT_JOIN_ELEMS, 0)
        idx.free()
