"""GPU parity of the search and tree options: exclude_self (row i without
i itself) against the oracle's lists minus the diagonal, and the octree
(b = 2 at every split, the classical octree the paper compares against)
against the oracle's octree build, leaf by leaf, and its lists."""
import numpy as np
import pytest

import oracle
from paper_1910_02639_amd import workloads as W
from tests.helpers import assert_same_lists, drop_self, gpu_lists, log, to_dev

pytestmark = pytest.mark.gpu

PRECS = ["fp32", "fp64"]


@pytest.fixture(scope="module", autouse=True)
def _setup():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    oracle.build(force=False)


def _lists(x, y, z, h, prec, **kw):
    import torch
    from paper_1910_02639_amd import btree
    dx, dy, dz, dh = to_dev(x, y, z, h)
    with btree.BTree(dx, dy, dz, precision=prec, **kw) as t:
        c, o, nb = t.find(dh)
        torch.cuda.synchronize()
        st = t.stats()
    return c.cpu().numpy().astype(np.int64), o.cpu().numpy(), nb.cpu().numpy(), st


def _excl_cases():
    rng = np.random.default_rng(31)
    out = [("U10k", W.uniform_cube(10_000, 0, 64.0), 64), ("P30k", W.plummer(30_000, 5), 32)]
    x, y, z = rng.normal(size=(3, 3000))
    h = rng.uniform(0.05, 0.4, 3000)
    h[::7] = 0.0
    h[::11] = 1e-300  # (2h)^2 underflows to 0: the row is empty, self included
    out.append(("random, zero and tiny h", (x, y, z, h), 16))
    # duplicates: every copy lists the others, not itself
    x = np.concatenate([np.full(200, 0.5), rng.random(800)])
    y = np.concatenate([np.full(200, 0.5), rng.random(800)])
    z = np.concatenate([np.full(200, 0.5), rng.random(800)])
    out.append(("duplicates", (x, y, z, np.full(1000, 0.03)), 16))
    # split levels and the exhaustive path
    x, y, z, h = W.uniform_cube(20_000, 7, 64.0)
    h = h.copy()
    h[::50] *= 1.6
    h[::997] *= 3.5
    out.append(("split paths", (x, y, z, h), 64))
    return out


@pytest.mark.parametrize("prec", PRECS)
def test_exclude_self_equals_oracle_minus_diagonal(prec):
    for name, (x, y, z, h), s in _excl_cases():
        log("exclude_self", name, prec)
        got = _lists(x, y, z, h, prec, bucket_size=s, exclude_self=True)
        want = drop_self(*oracle.lists(x, y, z, h))
        assert_same_lists(got, want)
        if name == "split paths":
            assert got[3]["split_items"] > 0 and got[3]["brute_chunks"] > 0


def test_exclude_self_batched():
    import torch
    from paper_1910_02639_amd import btree
    sets = [W.plummer(20_000, 41), W.uniform_cube(7_000, 42, 64.0), W.plummer(3_000, 43)]
    sizes = [len(s[0]) for s in sets]
    host = [np.concatenate([s[c] for s in sets]) for c in range(4)]
    dx, dy, dz, dh = to_dev(*host)
    for prec in PRECS:
        with btree.Batch(sizes, [dict(bucket_size=32), dict(bucket_size=64, octree=True),
                                 dict(bucket_size=16)], precision=prec,
                         exclude_self=True) as B:
            c, o, nb, totals = B.find(dx, dy, dz, dh)
            torch.cuda.synchronize()
            c, o, nb = c.cpu().numpy(), o.cpu().numpy(), nb.cpu().numpy()
        beg = 0
        for k, (x, y, z, h) in enumerate(sets):
            n = len(x)
            wc, wo, wn = drop_self(*oracle.lists(x, y, z, h))
            go = o[beg:beg + n + 1]
            assert np.array_equal(c[beg:beg + n], wc), (prec, k)
            assert np.array_equal(go - go[0], wo), (prec, k)
            assert np.array_equal(nb[go[0]:go[-1]], wn), (prec, k)
            assert totals[k] == wo[-1]
            beg += n


@pytest.mark.parametrize("name,s", [("U10k", 64), ("P60k", 32), ("P60k", 8), ("L1M", 128)])
def test_octree_matches_oracle_octree(name, s):
    """The device octree equals the oracle's (Algorithm 1 with b = 2 at every
    split), leaf by leaf, and is deeper than the b-tree on the same input."""
    from paper_1910_02639_amd import btree
    if name == "U10k":
        x, y, z, _ = W.uniform_cube(10_000, 0)
    elif name == "P60k":
        x, y, z, _ = W.plummer(60_000, 2)
    else:
        x, y, z, _ = W.lattice()
    log("octree", name, s)
    ref = oracle.build_tree(x, y, z, s=s, octree=True)
    dx, dy, dz = to_dev(x, y, z)
    with btree.BTree(dx, dy, dz, bucket_size=s, octree=True) as t:
        st = t.stats()
        ex = t.export()
    assert st["n_leaves"] == ref.n_leaves
    assert st["n_internal"] == ref.n_internal
    assert st["depth"] == ref.depth
    assert st["rounds"] == 0
    assert st["b_hist"] == {2: ref.n_internal}
    assert np.array_equal(ex["leaf_cnt"], ref.leaf_cnt)
    assert np.array_equal(ex["leaf_depth"], ref.leaf_depth)
    off = ref.leaf_offsets()
    order = ex["order"]
    for l in range(ref.n_leaves):
        a = np.sort(order[off[l]:off[l + 1]])
        assert np.array_equal(a, ref.members[off[l]:off[l + 1]]), l
    bt = oracle.build_tree(x, y, z, s=s)
    assert ref.depth >= bt.depth


@pytest.mark.parametrize("prec", PRECS)
def test_octree_lists(prec):
    for name, (x, y, z, h), s in [("U10k", W.uniform_cube(10_000, 1, 64.0), 32),
                                  ("P30k", W.plummer(30_000, 6), 16)]:
        log("octree lists", name, prec)
        got = _lists(x, y, z, h, prec, bucket_size=s, octree=True)
        assert_same_lists(got, oracle.lists(x, y, z, h))


def test_octree_and_exclude_self_p8m_all_rows():
    """P8M (8M-particle Plummer sphere) at the b-tree/octree comparison's
    bucket size: the octree's lists (depth 9) equal the oracle's row for
    row, and the b-tree's exclude_self lists equal them less each row's own
    index."""
    from tests.helpers import assert_all_rows
    x, y, z, h = W.plummer(8_000_000, 0)
    log("octree P8M")
    c, o, nb, st = _lists(x, y, z, h, "fp32", bucket_size=256, octree=True)
    log("octree P8M depth", st["depth"], "split", st["split_items"])
    assert st["depth"] > 3 and st["b_hist"] == {2: st["n_internal"]}
    assert_all_rows(x, y, z, h, c, o, nb, "octree P8M")
    log("exclude_self P8M")
    got = _lists(x, y, z, h, "fp32", bucket_size=256, beta=0.8, exclude_self=True)
    want = drop_self(c, o, nb)
    del c, o, nb
    assert_same_lists(got, want)
