"""Shared helpers of the GPU parity tests (no method arithmetic here)."""
import sys
import time

import numpy as np


def log(*a):
    print("[%s]" % time.strftime("%H:%M:%S"), *a, file=sys.stderr, flush=True)


def to_dev(*arrays):
    import torch
    return [torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to("cuda:0")
            for a in arrays]


def gpu_lists(x, y, z, h, precision="fp32", bucket_size=64, alpha=0.5, beta=0.5,
              max_depth=32):
    """Build + find on cuda:0; returns host (counts int64, offsets, nbrs, stats)."""
    from paper_1910_02639_amd import btree
    import torch
    dx, dy, dz, dh = to_dev(x, y, z, h)
    with btree.BTree(dx, dy, dz, bucket_size, alpha, beta, max_depth, precision) as t:
        c, o, nb = t.find(dh)
        torch.cuda.synchronize()
        st = t.stats()
    return (c.cpu().numpy().astype(np.int64), o.cpu().numpy(), nb.cpu().numpy(), st)


def assert_same_lists(got, want, rows=None):
    """Element-by-element equality of CSR lists (got from the GPU, want from
    the oracle restricted to `rows` when given)."""
    gc, go, gn = got[:3]
    wc, wo, wn = want
    if rows is None:
        assert np.array_equal(gc, wc), "counts differ at %s" % np.nonzero(gc != wc)[0][:10]
        assert np.array_equal(go, wo), "offsets differ"
        assert np.array_equal(gn, wn), "lists differ"
        return
    for k, i in enumerate(rows):
        a = gn[go[i]:go[i + 1]]
        b = wn[wo[k]:wo[k + 1]]
        assert gc[i] == wc[k], (i, gc[i], wc[k])
        assert np.array_equal(a, b), "row %d differs" % i


def check_csr_invariants(counts, offsets, nbrs, n):
    assert offsets[0] == 0
    assert np.array_equal(np.diff(offsets), counts)
    assert offsets[-1] == nbrs.shape[0]
    if nbrs.shape[0]:
        assert nbrs.min() >= 0 and nbrs.max() < n
    # rows strictly ascending: any non-increase must sit at a row boundary
    if nbrs.shape[0] > 1:
        bad = np.nonzero(np.diff(nbrs.astype(np.int64)) <= 0)[0] + 1
        starts = set(offsets[:-1].tolist())
        assert all(int(b) in starts for b in bad)


def assert_all_rows(x, y, z, h, counts, offsets, nbrs, what=""):
    """Every row of GPU lists against the oracle's cell list (the same
    definition as the brute force, pinned to it byte for byte), plus the
    CSR shape: offsets[0] = 0, offsets[n] = number of entries."""
    import oracle
    counts = np.ascontiguousarray(counts, dtype=np.int32)
    assert offsets[0] == 0, what
    assert offsets[-1] == nbrs.shape[0], what
    k, bad = oracle.cell_check(x, y, z, h, counts, offsets, nbrs)
    assert k == 0, "%s: %d rows differ from the oracle, first %s" % (what, k, bad[:10].tolist())


def drop_self(counts, offsets, nbrs):
    """CSR lists with every row's own index removed (j == i): the expected
    result of exclude_self, from lists that include it."""
    n = len(counts)
    rows = np.repeat(np.arange(n, dtype=np.int64), np.asarray(counts, dtype=np.int64))
    keep = nbrs.astype(np.int64) != rows
    c = np.bincount(rows[keep], minlength=n).astype(np.int64)
    o = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(c, out=o[1:])
    return c, o, nbrs[keep]
