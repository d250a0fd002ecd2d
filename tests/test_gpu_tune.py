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
        assert res["trials"] == 7
        assert res["path"] in (1, 2) and res["sort_items"] in (16, 32)
        assert res["path"] == 1 or res["group_cap"] in (1024, 2048, 4096)
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
            assert res["trials"] == 8 and res["batch_tile"] in (1 << 20, 1 << 21, 1 << 22, 1 << 23)
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
