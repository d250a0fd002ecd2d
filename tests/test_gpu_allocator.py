"""The allocator hook (sd_set_allocator): every device allocation of a context
comes from the provider, results stay equal to the oracle's, an allocation
failure anywhere in a call surfaces as SD_E_NOMEM with everything taken given
back and the context still usable, and releasing the context (or an index
built with the hook) returns every block."""
import ctypes

import numpy as np
import pytest

import cdr3gen

pytestmark = pytest.mark.gpu


def log(msg):
    print(msg, flush=True)


class Provider:
    """Device memory from PyTorch's caching allocator, counting what is out;
    fail_after = m makes the (m+1)-th and every later allocation fail."""

    def __init__(self, fail_after=None):
        import torch
        self.torch = torch
        self.out = {}
        self.calls = 0
        self.fail_after = fail_after

    def alloc(self, n):
        self.calls += 1
        if self.fail_after is not None and self.calls > self.fail_after:
            return None
        p = self.torch.cuda.caching_allocator_alloc(n, 0, self.torch.cuda.current_stream(0))
        assert p % 256 == 0
        self.out[p] = n
        return p

    def free(self, p):
        assert p in self.out, "a block the provider never handed out came back"
        del self.out[p]
        self.torch.cuda.caching_allocator_delete(p)


def to_dev(codes, offsets):
    import torch
    return (torch.from_numpy(np.ascontiguousarray(codes)).cuda(),
            torch.from_numpy(np.ascontiguousarray(offsets)).cuda())


def same(got, want):
    gi, gj, gd = [np.asarray(x) for x in got.numpy()]
    wi, wj, wd = want
    return (len(gi) == len(wi) and np.array_equal(gi.astype(np.uint32), wi)
            and np.array_equal(gj.astype(np.uint32), wj) and np.array_equal(gd.astype(np.int32), wd))


def test_torch_allocator_parity_10k():
    import oracle
    from paper_2403_09010_amd import Context
    c, o = cdr3gen.plain("plain_10k")
    prov = Provider()
    with Context(0) as ctx:
        ctx.set_allocator(prov.alloc, prov.free)
        for k in (1, 2):
            log(f"10K k={k} with device memory from the torch caching allocator")
            r = ctx.self_search(*to_dev(c, o), k)
            assert same(r, oracle.self_search(c, o, k))
        assert prov.calls > 10  # the scratch of the searches came from the provider
        # between calls only the context's own areas (look-back status, counters) stay out
        assert len(prov.out) <= 2
    assert prov.out == {}, "blocks still out after the context was released"


def test_use_torch_allocator_binding():
    import oracle
    import torch
    from paper_2403_09010_amd import Context
    c, o = cdr3gen.subset(*cdr3gen.plain("plain_1m"), 20000)
    before = torch.cuda.memory_allocated(0)
    with Context(0) as ctx:
        ctx.use_torch_allocator()
        r = ctx.self_search(*to_dev(c, o), 2)
        assert torch.cuda.memory_allocated(0) > before  # the context's areas are torch blocks
        assert same(r, oracle.self_search(c, o, 2))
    torch.cuda.synchronize()


@pytest.mark.parametrize("fail_after", [0, 3, 9, 25])
def test_null_allocation_is_nomem_and_leaks_nothing(fail_after):
    """Failure injection from the host: the provider returns NULL from its
    (fail_after+1)-th call on, at different points of a search."""
    import oracle
    from paper_2403_09010_amd import Context, SymdelError
    c, o = cdr3gen.plain("plain_10k")
    dc, do = to_dev(c, o)
    prov = Provider(fail_after=fail_after)
    ctx = Context(0)
    try:
        ctx.set_allocator(prov.alloc, prov.free)
        log(f"10K k=2 with allocation {fail_after + 1} failing")
        with pytest.raises(SymdelError) as e:
            ctx.self_search(dc, do, 2)
        assert e.value.name == "SD_E_NOMEM"
        assert len(prov.out) <= 2, f"{len(prov.out)} blocks still out after the failed call"
        # still usable: with a provider that works again the search is exact
        prov.fail_after = None
        assert same(ctx.self_search(dc, do, 2), oracle.self_search(c, o, 2))
    finally:
        ctx.close()
    assert prov.out == {}


def test_state_and_argument_errors():
    from paper_2403_09010_amd import Context, SymdelError
    from paper_2403_09010_amd.symdel import ALLOC_FN, FREE_FN, _Seqs
    c, o = cdr3gen.subset(*cdr3gen.plain("plain_10k"), 500)
    dc, do = to_dev(c, o)
    with Context(0) as ctx:
        # one function without the other is rejected
        rc = ctx._lib.sd_set_allocator(ctx._h, ALLOC_FN(lambda n, u: None), FREE_FN(), None)
        assert rc == -1
        # a device result still held by the caller blocks the switch
        s = _Seqs(dc.data_ptr(), do.data_ptr(), len(o) - 1, 1)
        import torch
        p = ctx.self_search_raw(s, 1, int(torch.cuda.current_stream().cuda_stream))
        prov = Provider()
        with pytest.raises(SymdelError) as e:
            ctx.set_allocator(prov.alloc, prov.free)
        assert e.value.name == "SD_E_STATE"
        ctx.free_pairs(p)
        ctx.set_allocator(prov.alloc, prov.free)
        ctx.self_search(dc, do, 1)
        ctx.set_allocator(None, None)  # back to the library's own pool
        assert prov.out == {}
        ctx.self_search(dc, do, 1)


def test_index_built_with_the_hook():
    import oracle
    from paper_2403_09010_amd import Context
    ref = cdr3gen.generate(21, 5000)
    qry = cdr3gen.generate_query(22, 800, *ref, ref_mut_frac=0.3)
    prov = Provider()
    with Context(0) as ctx:
        ctx.set_allocator(prov.alloc, prov.free)
        idx = ctx.build_index(*to_dev(*ref), 2)
        n_idx = len(prov.out)
        assert n_idx >= 4  # the index's arrays are provider blocks
        r = ctx.query(idx, *to_dev(*qry), 2)
        assert same(r, oracle.query_search(ref, qry, 2))
        idx.free()
        assert len(prov.out) <= 2
    assert prov.out == {}
