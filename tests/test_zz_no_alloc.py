"""The entry point that allocates nothing (sd_self_search_noalloc): through
the C ABI it returns exactly what sd_self_search returns on the same input,
on consecutive calls that reuse the fixed scratch area (the second smaller
than the first), without asking any allocator for memory; results that do
not fit the caller's arrays and inputs over the stated maximum fail with a
clear error and leave the context usable."""
import numpy as np
import pytest

import cdr3gen

pytestmark = pytest.mark.gpu


def log(msg):
    print(msg, flush=True)


def dev_inputs(codes, offsets):
    import torch
    return (torch.from_numpy(np.ascontiguousarray(codes)).cuda(),
            torch.from_numpy(np.ascontiguousarray(offsets)).cuda())


def outputs(cap):
    import torch
    return (torch.empty(cap, dtype=torch.int32, device="cuda"),
            torch.empty(cap, dtype=torch.int32, device="cuda"),
            torch.empty(cap, dtype=torch.uint8, device="cuda"))


def noalloc_triples(ctx, codes, offsets, k, cap):
    import torch
    oi, oj, od = outputs(cap)
    n = ctx.self_search_noalloc(*dev_inputs(codes, offsets), k, oi, oj, od)
    torch.cuda.synchronize()
    return (oi[:n].cpu().numpy().astype(np.uint32), oj[:n].cpu().numpy().astype(np.uint32),
            od[:n].cpu().numpy().astype(np.int32))


def plain_triples(ctx, codes, offsets, k):
    i, j, d = ctx.self_search(*dev_inputs(codes, offsets), k).numpy()
    return i.astype(np.uint32), j.astype(np.uint32), d.astype(np.int32)


def assert_same(got, want, what):
    assert len(got[0]) == len(want[0]), (what, len(got[0]), len(want[0]))
    for g, w in zip(got, want):
        assert np.array_equal(g, w), what


@pytest.mark.parametrize("k", [1, 2])
def test_noalloc_equals_self_search_on_consecutive_calls(k):
    from paper_2403_09010_amd import Context
    codes, offsets = cdr3gen.plain("plain_10k")
    with Context(0) as ctx:
        for n in (6000, 1500):  # the second call is smaller and reuses the area
            c, o = cdr3gen.subset(codes, offsets, n)
            log(f"noalloc k={k} n={n}")
            want = plain_triples(ctx, c, o, k)
            got = noalloc_triples(ctx, c, o, k, len(want[0]) + 64)
            assert_same(got, want, f"k={k} n={n}")
            log(f"  {len(want[0])} pairs equal")


def test_noalloc_asks_no_allocator():
    """With an allocator hook that refuses everything, the ordinary entry
    point fails and the no-allocation one still returns its result, without
    a single call to the hook."""
    from paper_2403_09010_amd import Context
    from paper_2403_09010_amd.symdel import SD_E_NOMEM, SymdelError
    codes, offsets = cdr3gen.subset(*cdr3gen.plain("plain_10k"), 3000)
    with Context(0) as ctx:
        want = plain_triples(ctx, codes, offsets, 2)
        calls = []
        ctx.set_allocator(lambda n: calls.append(n) or None, lambda p: None)
        with pytest.raises(SymdelError) as e:
            plain_triples(ctx, codes, offsets, 2)
        assert e.value.code == SD_E_NOMEM
        calls.clear()
        for _ in range(2):
            got = noalloc_triples(ctx, codes, offsets, 2, len(want[0]))
            assert_same(got, want, "hook refusing every allocation")
        assert calls == [], f"the no-allocation call asked the hook for {calls}"
        ctx.set_allocator(None, None)


def test_noalloc_errors_leave_the_context_usable():
    from paper_2403_09010_amd import Context
    from paper_2403_09010_amd.symdel import SD_E_NOMEM, SD_E_TOO_MANY, SymdelError
    codes, offsets = cdr3gen.subset(*cdr3gen.plain("plain_10k"), 2000)
    with Context(0) as ctx:
        want = plain_triples(ctx, codes, offsets, 2)
        assert len(want[0]) > 1
        # a result larger than the caller's arrays: the size needed comes back
        with pytest.raises(SymdelError) as e:
            noalloc_triples(ctx, codes, offsets, 2, len(want[0]) - 1)
        assert e.value.code == SD_E_NOMEM and e.value.needed == len(want[0])
        # more sequences than the stated maximum (rejected on the host)
        big_c, big_o = cdr3gen.subset(*cdr3gen.plain("plain_1m"), 16385)
        with pytest.raises(SymdelError) as e:
            noalloc_triples(ctx, big_c, big_o, 1, 16)
        assert e.value.code == SD_E_TOO_MANY
        got = noalloc_triples(ctx, codes, offsets, 2, len(want[0]))
        assert_same(got, want, "after the errors")
        # the ordinary entry point is unaffected by the fixed-area calls
        assert_same(plain_triples(ctx, codes, offsets, 2), want, "ordinary call afterwards")


def test_noalloc_at_the_maximum_size():
    import oracle
    from paper_2403_09010_amd import Context
    codes, offsets = cdr3gen.subset(*cdr3gen.plain("plain_1m"), 16384)
    a, b, d = oracle.self_search(codes, offsets, 2)
    with Context(0) as ctx:
        got = noalloc_triples(ctx, codes, offsets, 2, len(a) + 16)
    assert_same(got, (a, b, d), "16384 sequences, k=2, against the oracle")
    log(f"16384 sequences: {len(a)} pairs equal the oracle")
