"""Allocation failures forced from the host (the BTREE_FAULT_ALLOC hook):
every device allocation of a build and search, failed in turn, must come
back as BTREE_ENOMEM with its message, leave no half-made handle and no
leaked device memory, and the next clean call must give the oracle's lists."""
import os

import numpy as np
import pytest

import oracle
from paper_1910_02639_amd import workloads as W
from tests.helpers import assert_same_lists, log, to_dev

pytestmark = pytest.mark.gpu


def _device_free():
    import torch
    torch.cuda.synchronize()
    return torch.cuda.mem_get_info()[0]


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_each_allocation_failure_is_enomem(prec):
    from paper_1910_02639_amd import btree
    import torch
    x, y, z, h = W.uniform_cube(5000, 31, 64.0)
    dx, dy, dz, dh = to_dev(x, y, z, h)
    want = oracle.lists(x, y, z, h)
    free0 = _device_free()
    failed = 0
    try:
        for k in range(1, 200):
            os.environ["BTREE_FAULT_ALLOC"] = str(k)
            try:
                with btree.BTree(dx, dy, dz, bucket_size=32, precision=prec) as t:
                    c, o, nb = t.find(dh)
                    torch.cuda.synchronize()
            except btree.BTreeError as e:
                assert e.status == btree.BTREE_ENOMEM, str(e)
                assert "BTREE_FAULT_ALLOC" in str(e)
                failed += 1
                continue
            break  # k is past the last allocation: the whole call succeeded
        else:
            pytest.fail("more than 199 allocations")
    finally:
        del os.environ["BTREE_FAULT_ALLOC"]
    log("fault hook", prec, "allocations failed in turn:", failed)
    assert failed >= 5
    got = (c.cpu().numpy().astype(np.int64), o.cpu().numpy(), nb.cpu().numpy())
    assert_same_lists(got, want)
    # Handles of the failed calls were released: free memory is back
    # (within a margin for the allocator's own caching).
    del c, o, nb
    torch.cuda.empty_cache()
    assert _device_free() >= free0 - (64 << 20)
    # A clean call after the hook is unset.
    with btree.BTree(dx, dy, dz, bucket_size=32, precision=prec) as t:
        got = tuple(a.cpu().numpy() for a in t.find(dh))
    assert_same_lists((got[0].astype(np.int64), got[1], got[2]), want)
