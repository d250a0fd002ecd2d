"""Paired-chain records (the paper's Discussion: the CDR3s of both chains of
a receptor joined by a token that is never deleted): the GPU's paired self
search returns exactly the oracle's pairs, with d = Lev(a) + Lev(b) <= k,
on generated records, on exhaustive small-alphabet records and under the
grouping configurations that reach every branch."""
import itertools

import numpy as np
import pytest

import cdr3gen

pytestmark = pytest.mark.gpu

CONFIGS = {"auto": {}, "hashed_cap256": {"cap": 256}, "b20_counted_pairs": {"bits": 20, "pair_sort": 2}}


def log(msg):
    print(msg, flush=True)


def make_ctx(cfg):
    from paper_2403_09010_amd import Context
    from paper_2403_09010_amd.symdel import OPT_GROUP_BITS, OPT_GROUP_CAP, OPT_PAIR_SORT
    c = Context(0)
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


def gpu_paired(ctx, a, b, k):
    i, j, d = ctx.paired_self_search(to_dev(*a), to_dev(*b), k).numpy()
    return i.astype(np.uint32), j.astype(np.uint32), d.astype(np.int32)


def assert_same(got, want):
    assert len(got[0]) == len(want[0]), (len(got[0]), len(want[0]))
    for g, w in zip(got, want):
        assert np.array_equal(g, np.asarray(w).astype(g.dtype))


def csr(strings):
    offs = np.zeros(len(strings) + 1, dtype=np.int64)
    offs[1:] = np.cumsum([len(s) for s in strings])
    return np.frombuffer(b"".join(strings), dtype=np.uint8).copy(), offs


@pytest.mark.parametrize("k", [0, 1, 2, 3])
def test_paired_generator_records_match_oracle(cctx, k):
    import oracle
    a, b = cdr3gen.paired(21, 3000 if k < 3 else 1200)
    log(f"paired self search, {len(a[1]) - 1} records, k={k}, config={cctx.name}")
    got = gpu_paired(cctx, a, b, k)
    want = oracle.paired_self_search(a, b, k)
    assert_same(got, want)
    if k >= 1:
        assert len(got[0]) > 0


def test_paired_exhaustive_small_alphabet(cctx):
    import oracle
    chains = [bytes(t) for L in range(1, 4) for t in itertools.product(range(2), repeat=L)]
    recs = list(itertools.product(chains, chains))
    a = csr([x for x, _ in recs])
    b = csr([y for _, y in recs])
    for k in (1, 2):
        log(f"paired exhaustive 2-letter chains of length 1..3 ({len(recs)} records), k={k}")
        assert_same(gpu_paired(cctx, a, b, k), oracle.paired_self_search(a, b, k))


def test_paired_token_is_never_deleted(cctx):
    """Records whose concatenations agree but whose chains split differently
    ((AB, C) and (A, BC)) are not within distance 1: the join must align."""
    import oracle
    a = csr([bytes([0, 1]), bytes([0])])
    b = csr([bytes([2]), bytes([1, 2])])
    got = gpu_paired(cctx, a, b, 1)
    assert len(got[0]) == 0
    assert_same(gpu_paired(cctx, a, b, 2), oracle.paired_self_search(a, b, 2))


def test_paired_errors():
    from paper_2403_09010_amd import Context, SymdelError
    with Context(0) as ctx:
        a = csr([bytes([0, 1]), bytes([0])])
        b = csr([bytes([2])])
        with pytest.raises(SymdelError) as e:
            ctx.paired_self_search(to_dev(*a), to_dev(*b), 1)
        assert e.value.name == "SD_E_INVAL"
        b2 = csr([bytes([2]), bytes([25])])
        with pytest.raises(SymdelError) as e:
            ctx.paired_self_search(to_dev(*a), to_dev(*b2), 1)
        assert e.value.name == "SD_E_ALPHABET"
