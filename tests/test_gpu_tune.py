"""The autotuner picks among configurations that all return the same bytes;
after tuning, results still equal the oracle's."""
import numpy as np
import pytest

import cdr3gen

pytestmark = pytest.mark.gpu


def log(msg):
    print(msg, flush=True)


def triples(r):
    i, j, d = r.numpy()
    return list(zip(i.astype(np.int64).tolist(), j.astype(np.int64).tolist(),
                    d.astype(np.int64).tolist()))


def test_self_search_autotune_keeps_results():
    import oracle
    from paper_2403_09010_amd import Context
    c, o = cdr3gen.plain("plain_10k")
    want = oracle.self_search(c, o, 2)
    want = list(zip(*(x.tolist() for x in want)))
    with Context(0) as ctx:
        log("autotune self search on plain_10k, k=2")
        res = ctx.autotune([(c, o)], 2, reps=1)
        log(f"  chosen {res}")
        # stage 1: 6 hashed configurations and the full-key path; stage 2:
        # two pair sorts, and on the hashed path two hash-bit counts and (at
        # capacity 2048) the other grouping shape
        assert 9 <= res["trials"] <= 12 and res["from_cache"] == 0
        assert res["path"] in (1, 2) and res["sort_items"] in (16, 32)
        assert res["path"] == 1 or res["group_cap"] in (1024, 2048, 4096)
        assert res["pair_sort"] in (0, 1, 2) and res["group_shape"] in (0, 1)
        assert res["best_s"] > 0 and res["default_s"] > 0
        assert triples(ctx.self_search(c, o, 2, device_output=False)) == want


def test_query_autotune_keeps_results():
    from paper_2403_09010_amd import Context
    ref = cdr3gen.generate(61, 5000)
    sets = [cdr3gen.generate_query(62 + x, n, *ref, ref_mut_frac=0.2)
            for x, n in enumerate([300, 4000, 50, 1200])]
    with Context(0) as ctx:
        idx = ctx.build_index(*ref, 2)
        try:
            before = [triples(r) for r in ctx.query_batch(idx, sets, 2, device_output=False)]
            log("autotune query batches")
            res = ctx.autotune(sets, 2, index=idx, reps=1)
            log(f"  chosen {res}")
            assert res["trials"] == 9 and res["batch_tile"] in (1 << 20, 1 << 21, 1 << 22, 1 << 23)
            assert res["batch_graph"] in (0, 1)
            after = [triples(r) for r in ctx.query_batch(idx, sets, 2, device_output=False)]
            assert before == after
        finally:
            idx.free()


def test_autotune_rejects_bad_arguments():
    from paper_2403_09010_amd import Context, SymdelError
    c, o = cdr3gen.plain("plain_10k")
    with Context(0) as ctx:
        with pytest.raises(SymdelError):
            ctx.autotune([(c, o), (c, o)], 2)  # self search takes one sample
        with pytest.raises(SymdelError):
            ctx.autotune([(c, o)], 2, reps=0)
        assert len(ctx.self_search(c, o, 1, device_output=False)) > 0


def test_autotune_cache_round_trip(tmp_path):
    """A choice stored in the cache file is applied by a fresh context without
    trials, under a key of the architecture, the shape buckets and k; other
    keys are tuned and added; a file that does not parse is rewritten."""
    import json

    import oracle
    from paper_2403_09010_amd import Context
    c, o = cdr3gen.subset(*cdr3gen.plain("plain_10k"), 3000)
    path = str(tmp_path / "tune.json")
    with Context(0) as ctx:
        ctx.set_tune_cache(path)
        log("autotune with an empty cache file")
        first = ctx.autotune([(c, o)], 2, reps=1)
        assert first["from_cache"] == 0 and first["trials"] >= 9
    data = json.load(open(path))
    assert len(data) == 1
    (key, entry), = data.items()
    assert key.split("/")[1:] == ["self", "s11", "n0", "k2"], key
    assert key.split("/")[0].startswith("gfx")
    for name in ("path", "group_cap", "sort_items", "group_bits", "pair_sort", "group_shape"):
        assert entry[name] == first[name], name
    with Context(0) as ctx:
        ctx.set_tune_cache(path)
        log("autotune again: applied from the cache")
        again = ctx.autotune([(c, o)], 2, reps=1)
        assert again["from_cache"] == 1 and again["trials"] == 0
        for name in ("path", "group_cap", "sort_items", "group_bits", "pair_sort", "group_shape"):
            assert again[name] == first[name], name
        want = list(zip(*(x.tolist() for x in oracle.self_search(c, o, 2))))
        assert triples(ctx.self_search(c, o, 2, device_output=False)) == want
        log("autotune at k=1: a new key")
        k1 = ctx.autotune([(c, o)], 1, reps=1)
        assert k1["from_cache"] == 0
    data = json.load(open(path))
    assert len(data) == 2 and any(x.endswith("/k1") for x in data)
    with open(path, "w") as f:
        f.write("{not json")
    with Context(0) as ctx:
        ctx.set_tune_cache(path)
        log("autotune over a file that does not parse")
        res = ctx.autotune([(c, o)], 1, reps=1)
        assert res["from_cache"] == 0
        ctx.set_tune_cache(None)
    assert len(json.load(open(path))) == 1
