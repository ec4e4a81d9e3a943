"""chl_query_path_hops_noalloc: the path-length query that takes no device
memory from the allocator (its scratch is a fixed device array of the
library) gives what chl_query_path_hops gives, on two calls in a row, the
second with fewer pairs, and rejects more pairs than its array holds."""
import numpy as np
import pytest

import graphgen as gg

pytestmark = pytest.mark.gpu


def test_noalloc_path_hops_matches():
    import torch
    from paper_1907_00140_amd import chl
    al = chl.TorchAllocator()
    c = gg.make_config("rmat12s9")
    L = chl.build(c["row_ptr"], c["col"], c["w"], c["order"], allocator=al)
    par, slot = L.parents(c["row_ptr"], c["col"], c["w"])
    g = np.random.default_rng(5)
    for q in (60_000, 7_001):
        pairs = torch.from_numpy(g.integers(0, c["n"], size=(q, 2)).astype(np.int32)).cuda()
        want_h, want_o = L.path_hops(pairs, par, slot)
        torch.cuda.synchronize()
        hops = torch.full((q,), -7, dtype=torch.int64, device="cuda")
        off = torch.full((q + 1,), -7, dtype=torch.int64, device="cuda")
        before = al.calls
        got_h, got_o = L.path_hops(pairs, par, slot, noalloc=True, out=(hops, off))
        torch.cuda.synchronize()
        assert al.calls == before, "the no-alloc call allocated"
        assert torch.equal(got_h, want_h) and torch.equal(got_o, want_o), q
        # the paths written from these offsets equal the allocating call's
        _, _, path = L.paths(pairs, par, slot)
        assert int(got_o[-1].item()) == path.numel()
    big = torch.zeros((chl.NOALLOC_MAX_PAIRS + 1, 2), dtype=torch.int32, device="cuda")
    with pytest.raises(chl.ChlError) as e:
        L.path_hops(big, par, slot, noalloc=True)
    assert e.value.code == -1
    L.free()
