"""Host-side staging of inputs: a large host set goes to the device in
pinned pieces (its distances on sampled pairs equal the oracle's, and its
self search equals the same set's from device memory), batches mix host and
device sets (each set equal to the oracle's query of it alone, eager and as
a captured graph), and bad offsets are refused before any kernel runs, with
the context usable afterwards."""
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


def triples(r):
    i, j, d = r.numpy()
    return list(zip(i.astype(np.int64).tolist(), j.astype(np.int64).tolist(),
                    d.astype(np.int64).tolist()))


def oracle_query(ref, qry, k):
    import oracle
    if len(qry[1]) <= 1:
        return []
    a, b, d = oracle.query_search(ref, qry, k)
    return list(zip(a.tolist(), b.tolist(), d.tolist()))


@pytest.fixture(scope="module")
def ctx():
    from paper_2403_09010_amd import Context
    c = Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def big():
    # 300,000 sequences: about 4.5 MB of codes and 2.4 MB of offsets, so the
    # host staging takes several pieces of each
    return cdr3gen.generate(31, 300_000)


def test_large_host_set_distances_equal_the_oracle(ctx, big):
    import torch
    import oracle
    codes, offs = big
    n = len(offs) - 1
    rng = np.random.default_rng(3)
    ia = rng.integers(0, n, 3000)
    ib = rng.integers(0, n, 3000)
    ia[:2] = [0, n - 1]
    ib[:2] = [n - 1, n // 2]
    log(f"sd_pair_distance on {len(ia)} sampled pairs of a {n}-sequence host set")
    d = ctx.pair_distance((codes, offs), (codes, offs),
                          torch.from_numpy(ia.astype(np.int32)).cuda(),
                          torch.from_numpy(ib.astype(np.int32)).cuda()).cpu().numpy()

    def seq(x):
        return codes[offs[x]:offs[x + 1]].tobytes()
    want = np.array([oracle.lev(seq(a), seq(b)) for a, b in zip(ia, ib)])
    assert np.array_equal(d.astype(np.int64), want)


def test_large_host_set_search_equals_device_input(ctx, big):
    log("self search of the 300K set, k=1: host input and host output against device input")
    h = ctx.self_search(*big, 1, device_output=False)
    d = ctx.self_search(*to_dev(*big), 1, device_output=True)
    for a, b in zip(h.numpy(), d.numpy()):
        assert np.array_equal(a, b)
    assert len(h) > 0


def test_host_offsets_refused(ctx, big):
    from paper_2403_09010_amd import SymdelError
    codes, offs = big
    bad = offs.copy()
    bad[250_000] = bad[249_999] - 1
    log("a decreasing offset deep in a large host set")
    with pytest.raises(SymdelError) as e:
        ctx.self_search(codes, bad, 1)
    assert e.value.name == "SD_E_INVAL"
    bad = offs.copy()
    bad[0] = 3
    with pytest.raises(SymdelError) as e:
        ctx.self_search(codes, bad, 1)
    assert e.value.name == "SD_E_INVAL"
    log("the context still searches")
    small = cdr3gen.plain("plain_10k")
    import oracle
    a, b, dd = oracle.self_search(*small, 1)
    r = ctx.self_search(*small, 1, device_output=False)
    i, j, d = r.numpy()
    assert np.array_equal(i, a) and np.array_equal(j, b) and np.array_equal(d, dd)


@pytest.mark.parametrize("graph", [0, 1])
def test_mixed_host_and_device_sets(ctx, graph):
    from paper_2403_09010_amd.symdel import OPT_BATCH_GRAPH, OPT_BATCH_TILE
    ref = cdr3gen.generate(11, 3000)
    sizes = [700, 0, 1800, 45, 2600, 310]
    sets = [cdr3gen.generate_query(900 + x, s, *ref, ref_mut_frac=0.25) if s else
            (np.zeros(0, np.uint8), np.zeros(1, np.int64)) for x, s in enumerate(sizes)]
    # even sets from device memory, odd ones from host memory
    args = [to_dev(*s) if x % 2 == 0 else s for x, s in enumerate(sets)]
    idx = ctx.build_index(*to_dev(*ref), 2)
    try:
        ctx.set_option(OPT_BATCH_GRAPH, graph)
        ctx.set_option(OPT_BATCH_TILE, 2000)  # sets split across tiles in the graph
        log(f"mixed batch of {len(sets)} sets, graph={graph}")
        for rep in range(2):
            outs = ctx.query_batch(idx, args, 2, device_output=False)
            for x, (s, o) in enumerate(zip(sets, outs)):
                assert triples(o) == oracle_query(ref, s, 2), f"set {x}, call {rep}"
    finally:
        ctx.set_option(OPT_BATCH_GRAPH, 0)
        ctx.set_option(OPT_BATCH_TILE, 0)
        idx.free()


@pytest.mark.parametrize("graph", [0, 1])
def test_batch_offsets_refused(ctx, graph):
    from paper_2403_09010_amd import SymdelError
    from paper_2403_09010_amd.symdel import OPT_BATCH_GRAPH
    ref = cdr3gen.generate(11, 3000)
    good = cdr3gen.generate_query(77, 400, *ref, ref_mut_frac=0.25)
    codes, offs = good
    dec = offs.copy()
    dec[200] = dec[199] - 1
    empty_seq = offs.copy()
    empty_seq[300] = empty_seq[299]
    idx = ctx.build_index(*to_dev(*ref), 2)
    try:
        ctx.set_option(OPT_BATCH_GRAPH, graph)
        log(f"batch with a decreasing offset in a device set, graph={graph}")
        with pytest.raises(SymdelError) as e:
            ctx.query_batch(idx, [to_dev(*good), to_dev(codes, dec)], 2)
        assert e.value.name == "SD_E_INVAL"
        log("batch with a sequence of length 0")
        with pytest.raises(SymdelError) as e:
            ctx.query_batch(idx, [good, (codes, empty_seq)], 2)
        assert e.value.name == "SD_E_LENGTH"
        log("the context still answers the good set")
        outs = ctx.query_batch(idx, [good, to_dev(*good)], 2, device_output=False)
        want = oracle_query(ref, good, 2)
        assert triples(outs[0]) == want and triples(outs[1]) == want
    finally:
        ctx.set_option(OPT_BATCH_GRAPH, 0)
        idx.free()
