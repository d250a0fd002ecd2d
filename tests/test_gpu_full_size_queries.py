"""The batched and served workloads at their full sizes, checked against the
oracle on sampled queries: for each sampled query sequence, its neighbours
in the GPU result equal every reference within the distance, found by the
oracle's one-to-many distance over the whole reference (and, for weighted
serving, the oracle's weighted score of those); every reported distance of
the sampled sets is the oracle's. The eager tiles and the captured graph give
the same bytes for every set."""
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import cdr3gen

pytestmark = pytest.mark.gpu


def log(msg):
    print(msg, flush=True)


def to_dev(codes, offsets):
    import torch
    return (torch.from_numpy(np.ascontiguousarray(codes)).cuda(),
            torch.from_numpy(np.ascontiguousarray(offsets)).cuda())


def triples(p):
    i, j, d = p.numpy()
    return i.astype(np.int64), j.astype(np.int64), d.astype(np.int64)


def seq(codes, offsets, x):
    return codes[offsets[x]:offsets[x + 1]].tobytes()


def neighbours_by_oracle(ref, queries, k):
    """{query index: (ref ids, distances)} of every reference within k."""
    import oracle

    def one(q):
        d = oracle.lev_one_to_many(q, *ref)
        r = np.nonzero(d <= k)[0]
        return r.astype(np.int64), d[r].astype(np.int64)

    with ThreadPoolExecutor(max_workers=oracle.host_threads()) as ex:
        return list(ex.map(one, queries))


def check_sampled(got, qset, ref, picks, k):
    """The GPU neighbours of the picked queries equal the oracle's; every
    reported distance of the set is the oracle's (on up to 3,000 pairs)."""
    import oracle
    i, j, d = got
    assert np.all(np.diff(i) >= 0) and np.all((np.diff(i) > 0) | (np.diff(j) > 0))
    want = neighbours_by_oracle(ref, [seq(*qset, q) for q in picks], k)
    for q, (wr, wd) in zip(picks, want):
        lo, hi = np.searchsorted(i, [q, q + 1])
        assert np.array_equal(j[lo:hi], wr), f"query {q}"
        assert np.array_equal(d[lo:hi], wd), f"query {q}"
    rng = np.random.default_rng(len(i))
    for x in rng.choice(len(i), min(len(i), 3000), replace=False) if len(i) else []:
        assert oracle.lev(seq(*qset, i[x]), seq(*ref, j[x])) == d[x]


def test_batched_512_sets_against_2m_sampled():
    from paper_2403_09010_amd import Context
    from paper_2403_09010_amd.symdel import OPT_BATCH_GRAPH
    p = cdr3gen.BATCHED
    ref = cdr3gen.generate(p["ref_seed"], p["ref_n"])
    sets = cdr3gen.batched_sets(ref, p["sets"])
    log(f"512 sets, {sum(len(o) - 1 for _, o in sets)} query sequences, against 2M")
    dsets = [to_dev(*s) for s in sets]
    with Context(0) as ctx:
        idx = ctx.build_index(*to_dev(*ref), 2)
        try:
            eager = [triples(o) for o in ctx.query_batch(idx, dsets, 2)]
            ctx.set_option(OPT_BATCH_GRAPH, 1)
            log("the same batch as a captured graph")
            graph = [triples(o) for o in ctx.query_batch(idx, dsets, 2)]
            ctx.set_option(OPT_BATCH_GRAPH, 0)
        finally:
            idx.free()
    assert sum(len(e[0]) for e in eager) == 6_867_721
    for x, (e, g) in enumerate(zip(eager, graph)):
        assert all(np.array_equal(a, b) for a, b in zip(e, g)), f"set {x}: graph differs"
    rng = np.random.default_rng(17)
    for x in sorted(rng.choice(len(sets), 6, replace=False).tolist()):
        n = len(sets[x][1]) - 1
        # three sampled queries, one of them with neighbours when the set has any
        picks = set(rng.choice(n, 2, replace=False).tolist())
        if len(eager[x][0]):
            picks.add(int(eager[x][0][rng.integers(len(eager[x][0]))]))
        log(f"set {x} ({n} sequences): queries {sorted(picks)} against the oracle")
        check_sampled(eager[x], sets[x], ref, sorted(picks), 2)


def test_served_5m_weighted_sampled():
    import oracle
    from paper_2403_09010_amd import Context, Server
    p = cdr3gen.SERVED
    ref = cdr3gen.generate(p["ref_seed"], p["ref_n"])
    subst = cdr3gen.cost_matrix(p["cost_seed"], p["cost_lo"], p["cost_hi"])
    sizes = cdr3gen.loguniform_sizes(p["arrival_seed"], 12, 100, 3000)
    reqs = [cdr3gen.generate_query(30000 + x, int(n), *ref, ref_mut_frac=0.2)
            for x, n in enumerate(sizes)]
    log(f"12 weighted requests against the 5M reference")
    with Context(0) as ctx:
        idx = ctx.build_index(*to_dev(*ref), 2)
        try:
            with Server(idx, k=2, workers=2, subst=subst, indel=p["indel"],
                        max_score=p["max_score"]) as sv:
                ids = [sv.submit(*r) for r in reqs]
                got = [triples(sv.poll(r, timeout_ms=120000)[0]) for r in ids]
        finally:
            idx.free()
    rng = np.random.default_rng(23)
    for x in (0, 5, 11):
        i, j, d = got[x]
        n = len(reqs[x][1]) - 1
        picks = set(rng.choice(n, 2, replace=False).tolist())
        if len(i):
            picks.add(int(i[rng.integers(len(i))]))
        picks = sorted(picks)
        # weighted score <= 8 implies Levenshtein <= 2, so the oracle's
        # Levenshtein neighbours hold every weighted one
        lev = neighbours_by_oracle(ref, [seq(*reqs[x], q) for q in picks], 2)
        log(f"request {x} ({n} sequences): queries {picks} against the oracle")
        for q, (r, _) in zip(picks, lev):
            score = np.array([oracle.weighted(seq(*reqs[x], q), seq(*ref, t), subst, p["indel"])
                              for t in r], dtype=np.int64)
            keep = score <= p["max_score"]
            lo, hi = np.searchsorted(i, [q, q + 1])
            assert np.array_equal(j[lo:hi], r[keep]), f"request {x} query {q}"
            assert np.array_equal(d[lo:hi], score[keep]), f"request {x} query {q}"
