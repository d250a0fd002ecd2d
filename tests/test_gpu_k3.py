"""Three deletions (k = 3; the paper's Fig. 2C distance 3 and Section III D's
d = 3 prefilter): the hashed path enumerates every deletion set of up to
three positions (distinct strings once each) and returns exactly the
oracle's pairs, under the grouping and pair-sort configurations that reach
every branch at small size; query search against an index built at k = 3
matches the oracle's query search."""
import itertools

import numpy as np
import pytest

import cdr3gen

pytestmark = pytest.mark.gpu

CONFIGS = {
    "auto": {},
    "hashed_cap256": {"path": 2, "cap": 256},
    "hashed_1024_b20_counted_pairs": {"path": 2, "cap": 1024, "bits": 20, "pair_sort": 2},
    "hashed_fallback": {"path": 2, "cap": 256, "bits": 4},
}


def log(msg):
    print(msg, flush=True)


def make_ctx(cfg):
    from paper_2403_09010_amd import Context
    from paper_2403_09010_amd.symdel import (OPT_GROUP_BITS, OPT_GROUP_CAP, OPT_PAIR_SORT,
                                             OPT_PATH)
    c = Context(0)
    c.set_option(OPT_PATH, cfg.get("path", 0))
    c.set_option(OPT_GROUP_CAP, cfg.get("cap", 0))
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


def gpu_triples(ctx, codes, offsets, k):
    i, j, d = ctx.self_search(*to_dev(codes, offsets), k).numpy()
    return i.astype(np.uint32), j.astype(np.uint32), d.astype(np.int32)


def oracle_triples(codes, offsets, k):
    import oracle
    return oracle.self_search_sharded(codes, offsets, k, threads=oracle.host_threads())


def assert_same(got, want):
    assert len(got[0]) == len(want[0]), (len(got[0]), len(want[0]))
    for g, w in zip(got, want):
        assert np.array_equal(g, np.asarray(w).astype(g.dtype))


def csr(strings):
    offs = np.zeros(len(strings) + 1, dtype=np.int64)
    offs[1:] = np.cumsum([len(s) for s in strings])
    return np.frombuffer(b"".join(strings), dtype=np.uint8).copy(), offs


def test_generator_subset_k3_matches_oracle(cctx):
    c, o = cdr3gen.subset(*cdr3gen.plain("plain_10k"), 4000)
    log(f"k=3 self search, first 4000 of plain_10k, config={cctx.name}")
    got = gpu_triples(cctx, c, o, 3)
    want = oracle_triples(c, o, 3)
    assert_same(got, want)
    assert (got[2] == 3).sum() > 0, "no pair at distance 3"
    log(f"  {len(got[0])} pairs")


def test_exhaustive_small_alphabet_k3(cctx):
    strings = [bytes(t) for L in range(1, 7) for t in itertools.product(range(3), repeat=L)]
    c, o = csr(strings)
    log(f"k=3 exhaustive 3-letter strings of length 1..6, config={cctx.name}")
    assert_same(gpu_triples(cctx, c, o, 3), oracle_triples(c, o, 3))


def test_runs_and_periodic_strings_k3(cctx):
    # repeated residues and short periods: most deletion triples repeat a
    # string, so only the canonical sets may be generated
    rng = np.random.default_rng(9)
    strings = []
    for _ in range(1500):
        L = int(rng.integers(1, 25))
        period = int(rng.integers(1, 4))
        motif = rng.integers(0, 3, period)
        s = np.resize(motif, L).astype(np.uint8)
        flips = rng.integers(0, L, int(rng.integers(0, 3)))
        s[flips] = rng.integers(0, 20, len(flips))
        strings.append(s.tobytes())
    c, o = csr(strings)
    log(f"k=3 runs and periods, 1500 strings, config={cctx.name}")
    assert_same(gpu_triples(cctx, c, o, 3), oracle_triples(c, o, 3))


def test_full_key_path_rejects_k3():
    from paper_2403_09010_amd import SymdelError
    ctx = make_ctx({"path": 1})
    try:
        c, o = cdr3gen.subset(*cdr3gen.plain("plain_10k"), 100)
        with pytest.raises(SymdelError) as e:
            ctx.self_search(*to_dev(c, o), 3)
        assert e.value.name == "SD_E_INVAL"
        # the context stays usable
        assert len(ctx.self_search(*to_dev(c, o), 1)) >= 0
    finally:
        ctx.close()


def test_query_k3_matches_oracle():
    import oracle
    from paper_2403_09010_amd import Context
    ref = cdr3gen.subset(*cdr3gen.plain("plain_10k"), 3000)
    qry = cdr3gen.generate(501, 800)
    with Context(0) as ctx:
        idx = ctx.build_index(*to_dev(*ref), 3)
        try:
            for k in (3, 2):
                log(f"query 800 against a k=3 index of 3000, k={k}")
                i, j, d = ctx.query(idx, *to_dev(*qry), k).numpy()
                a, b, e = oracle.query_search(ref, qry, k)
                assert_same((i.astype(np.uint32), j.astype(np.uint32), d.astype(np.int32)),
                            (a, b, e))
        finally:
            idx.free()
