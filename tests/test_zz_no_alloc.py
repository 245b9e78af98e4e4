"""The entry point that allocates no device memory
(btree_find_neighbors_noalloc) against btree_build + btree_find_neighbors,
element by element, on calls in a row: the second call is smaller than the
first, so contents the first left in the shared scratch must not leak into
its result; a third repeats the first."""
import numpy as np
import pytest

from paper_1910_02639_amd import workloads as W
from tests.helpers import log, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _setup():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"


def _reference(x, y, z, h, **kw):
    import torch
    from paper_1910_02639_amd import btree
    dx, dy, dz, dh = to_dev(x, y, z, h)
    with btree.BTree(dx, dy, dz, **kw) as t:
        c, o, nb = t.find(dh)
        torch.cuda.synchronize()
        return c.cpu().numpy(), o.cpu().numpy(), nb.cpu().numpy()


def _noalloc(x, y, z, h, cap, **kw):
    import torch
    from paper_1910_02639_amd import btree
    dx, dy, dz, dh = to_dev(x, y, z, h)
    n = len(x)
    counts = torch.full((n,), -7, dtype=torch.int32, device="cuda:0")
    offsets = torch.full((n + 1,), -7, dtype=torch.int64, device="cuda:0")
    nbrs = torch.full((cap + 16,), -7, dtype=torch.int32, device="cuda:0")
    total = btree.find_neighbors_noalloc(dx, dy, dz, dh, counts, offsets, nbrs[:cap], **kw)
    nb = nbrs.cpu().numpy()
    assert np.all(nb[total:] == -7), "entries written past the total"
    return counts.cpu().numpy(), offsets.cpu().numpy(), nb[:total]


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_noalloc_equals_build_and_find(prec):
    cases = [(W.plummer(60_000, 21), 32), (W.uniform_cube(9_000, 22, 64.0), 64),
             (W.plummer(60_000, 21), 32)]
    for k, ((x, y, z, h), s) in enumerate(cases):
        log("no-alloc call", k, "n", len(x), "s", s, prec)
        want = _reference(x, y, z, h, bucket_size=s, precision=prec)
        got = _noalloc(x, y, z, h, len(want[2]) + 100, bucket_size=s, precision=prec)
        assert np.array_equal(got[0], want[0]), "counts differ (call %d)" % k
        assert np.array_equal(got[1], want[1]), "offsets differ (call %d)" % k
        assert np.array_equal(got[2], want[2]), "lists differ (call %d)" % k


def test_noalloc_errors():
    import torch
    from paper_1910_02639_amd import btree
    x, y, z, h = W.uniform_cube(5_000, 23, 64.0)
    dx, dy, dz, dh = to_dev(x, y, z, h)
    counts = torch.zeros(5_000, dtype=torch.int32, device="cuda:0")
    offsets = torch.zeros(5_001, dtype=torch.int64, device="cuda:0")
    want = _reference(x, y, z, h)
    # capacity below the total: counts and offsets written, nbrs untouched
    small = torch.full((10,), -7, dtype=torch.int32, device="cuda:0")
    with pytest.raises(btree.BTreeError) as ei:
        btree.find_neighbors_noalloc(dx, dy, dz, dh, counts, offsets, small)
    assert ei.value.status == btree.BTREE_EOVERFLOW
    assert ei.value.total == len(want[2])
    assert np.array_equal(counts.cpu().numpy(), want[0])
    assert np.array_equal(offsets.cpu().numpy(), want[1])
    assert bool((small == -7).all())
    # above the size limit: rejected before any device work
    big = torch.zeros(btree.NOALLOC_MAX_N + 1, dtype=torch.float64, device="cuda:0")
    cb = torch.zeros(btree.NOALLOC_MAX_N + 1, dtype=torch.int32, device="cuda:0")
    ob = torch.zeros(btree.NOALLOC_MAX_N + 2, dtype=torch.int64, device="cuda:0")
    with pytest.raises(btree.BTreeError) as ei:
        btree.find_neighbors_noalloc(big, big, big, big, cb, ob, None)
    assert ei.value.status == btree.BTREE_EINVAL
    # empty input
    e = torch.zeros(0, dtype=torch.float64, device="cuda:0")
    o1 = torch.full((1,), 5, dtype=torch.int64, device="cuda:0")
    assert btree.find_neighbors_noalloc(e, e, e, e, torch.zeros(0, dtype=torch.int32,
                                                               device="cuda:0"), o1, None) == 0
    assert int(o1[0]) == 0
