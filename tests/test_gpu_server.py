"""The continuous-batching server: every request's result in the mix equals
the oracle's query result for that set (Levenshtein, or the weighted score),
equals the same set queried alone (bit-identical), and cancellation / budget
rejection behave as documented."""
import threading
import time

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
    return cdr3gen.generate(21, 20000)


@pytest.fixture(scope="module")
def index(ctx, ref):
    idx = ctx.build_index(*ref, 2)
    yield idx
    idx.free()


def same(a, b):
    ai, aj, ad = a.numpy()
    bi, bj, bd = b.numpy()
    return (np.array_equal(ai.astype(np.uint32), bi.astype(np.uint32))
            and np.array_equal(aj.astype(np.uint32), bj.astype(np.uint32))
            and np.array_equal(ad.astype(np.uint8), bd.astype(np.uint8)))


def make_requests(ref, count, seed):
    sizes = cdr3gen.loguniform_sizes(seed, count, 100, 5000)
    return [cdr3gen.generate_query(seed * 1000 + x, int(n), *ref, ref_mut_frac=0.2)
            for x, n in enumerate(sizes)]


def oracle_per_request(ref, reqs, subst=None):
    """The oracle's (q, r, d) for every request: one oracle query over the
    concatenated requests (a query's result does not depend on the others),
    split by request and with q made local to it."""
    import oracle
    codes = np.concatenate([c for c, _ in reqs])
    offs = [np.zeros(1, np.int64)]
    base, n = 0, [0]
    for c, o in reqs:
        offs.append(o[1:] + base)
        base += int(o[-1])
        n.append(n[-1] + len(o) - 1)
    offs = np.concatenate(offs)
    if subst is None:
        a, b, d = oracle.query_search(ref, (codes, offs), 2)
    else:
        a, b, d = oracle.query_weighted(ref, (codes, offs), subst, 8, 8)
    out = []
    for x in range(len(reqs)):
        lo, hi = np.searchsorted(a, [n[x], n[x + 1]])
        out.append(((a[lo:hi] - n[x]).astype(np.uint32), b[lo:hi].astype(np.uint32),
                    d[lo:hi].astype(np.int32)))
    return out


def equals_oracle(got, want):
    gi, gj, gd = got.numpy()
    wi, wj, wd = want
    return (len(gi) == len(wi) and np.array_equal(gi.astype(np.uint32), wi)
            and np.array_equal(gj.astype(np.uint32), wj)
            and np.array_equal(gd.astype(np.int32), wd))


def test_results_in_the_mix_equal_alone_and_oracle(ctx, ref, index):
    from paper_2403_09010_amd import Server
    reqs = make_requests(ref, 40, 7)
    want = oracle_per_request(ref, reqs)
    alone = [ctx.query(index, *r, 2, device_output=False) for r in reqs]
    log("server: 40 requests from two submitting threads, 3 workers")
    with Server(index, k=2, workers=3) as sv:
        ids = [None] * len(reqs)

        def submit(part):
            for x in part:
                ids[x] = sv.submit(*reqs[x])
                time.sleep(0.0005 * (x % 3))

        threads = [threading.Thread(target=submit, args=(range(p, len(reqs), 2),)) for p in (0, 1)]
        for t in threads:
            t.start()
        for t in threads:
            t.join()
        for x, rid in enumerate(ids):
            got, lat = sv.poll(rid, timeout_ms=60000)
            assert equals_oracle(got, want[x]), f"request {x} differs from the oracle"
            assert same(got, alone[x]), f"request {x}"
            assert lat > 0
        st = sv.stats()
    assert st["requests"] == len(reqs)
    assert st["batches"] <= len(reqs)
    log(f"server stats {st}")


def test_batches_really_merge(ctx, ref, index):
    from paper_2403_09010_amd import Server
    reqs = make_requests(ref, 24, 8)
    want = oracle_per_request(ref, reqs)
    # one worker: everything queued while the first batch runs joins the next
    with Server(index, k=2, workers=1) as sv:
        ids = [sv.submit(*r) for r in reqs]
        res = [sv.poll(i, timeout_ms=60000)[0] for i in ids]
        st = sv.stats()
    for x, (r, got) in enumerate(zip(reqs, res)):
        assert equals_oracle(got, want[x]), f"request {x} differs from the oracle"
        assert same(got, ctx.query(index, *r, 2, device_output=False))
    assert st["max_batch"] > 1 and st["batches"] < len(reqs)


def test_weighted_serving(ctx, ref, index):
    from paper_2403_09010_amd import Server
    subst = cdr3gen.cost_matrix()
    reqs = make_requests(ref, 10, 9)
    want = oracle_per_request(ref, reqs, subst=subst)
    assert sum(len(w[0]) for w in want) > 0
    with Server(index, k=2, workers=2, subst=subst, indel=8, max_score=8) as sv:
        ids = [sv.submit(*r) for r in reqs]
        for x, (r, rid) in enumerate(zip(reqs, ids)):
            got, _ = sv.poll(rid, timeout_ms=60000)
            assert equals_oracle(got, want[x]), f"weighted request {x} differs from the oracle"
            assert same(got, ctx.query_weighted(index, *r, subst, 8, 8, device_output=False))


def test_cancel_and_budget(ctx, ref, index):
    from paper_2403_09010_amd import Server, SymdelError
    reqs = make_requests(ref, 6, 10)
    with Server(index, k=2, workers=1) as sv:
        ids = [sv.submit(*r) for r in reqs]
        rc = sv.cancel(ids[-1])
        if rc == 0:
            with pytest.raises(SymdelError) as e:
                sv.poll(ids[-1], timeout_ms=60000)
            assert e.value.name == "SD_E_CANCELLED"
        else:  # it had already finished
            sv.poll(ids[-1], timeout_ms=60000)
        for rid in ids[:-1]:
            sv.poll(rid, timeout_ms=60000)
        with pytest.raises(SymdelError):
            sv.poll(ids[0], timeout_ms=0)  # a result is returned once
    with Server(index, k=2, workers=1, hbm_budget=1 << 16) as sv:
        rid = sv.submit(*reqs[0])
        with pytest.raises(SymdelError) as e:
            sv.poll(rid, timeout_ms=60000)
        assert e.value.name == "SD_E_NOMEM"


def test_destroy_with_pending_requests(ref, index):
    from paper_2403_09010_amd import Server
    reqs = make_requests(ref, 12, 11)
    sv = Server(index, k=2, workers=1)
    for r in reqs:
        sv.submit(*r)
    sv.close()  # queued requests are cancelled; the call returns
