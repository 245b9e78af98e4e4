"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Neighbour counts and lists are integers and must be equal element by
element, for both arithmetic forms (FP64 and FP32 filter + FP64 band).
"""
import numpy as np
import pytest

import oracle
from paper_1910_02639_amd import workloads as W
from tests.helpers import (assert_all_rows, assert_same_lists, check_csr_invariants, gpu_lists,
                           log, to_dev)

pytestmark = pytest.mark.gpu

PRECS = ["fp32", "fp64"]


@pytest.fixture(scope="module", autouse=True)
def _setup():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    oracle.build(force=False)


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_uniform_10k_full(prec, seed):
    x, y, z, h = W.uniform_cube(10_000, seed, 64.0)
    log("U10k seed", seed, prec)
    got = gpu_lists(x, y, z, h, prec, bucket_size=64)
    want = oracle.lists(x, y, z, h)
    assert_same_lists(got, want)
    st = got[3]
    assert st["brute_chunks"] == 0
    assert st["total"] == want[0].sum()


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("n,s", [(1, 64), (2, 1), (63, 64), (64, 64), (65, 64), (300, 8),
                                 (2000, 16), (5000, 128), (4097, 32)])
def test_small_random_full(prec, n, s):
    rng = np.random.default_rng(1000 + n + s)
    x, y, z = rng.normal(size=(3, n))
    h = rng.uniform(0.05, 0.4, n)
    h[::7] = 0.0  # some empty rows
    log("small", n, s, prec)
    got = gpu_lists(x, y, z, h, prec, bucket_size=s)
    want = oracle.lists(x, y, z, h)
    assert_same_lists(got, want)


@pytest.mark.parametrize("prec", PRECS)
def test_plummer_small_full(prec):
    x, y, z, h = W.plummer(30_000, 5)
    log("plummer 30k", prec)
    got = gpu_lists(x, y, z, h, prec, bucket_size=32)
    want = oracle.lists(x, y, z, h)
    assert_same_lists(got, want)
    log("plummer 30k exhaustive", got[3]["brute_chunks"], "split", got[3]["split_items"])
    # At n = 3e4 the outermost particles have 2h ~ 7 (h grows as rho^-1/3),
    # so their work items see most of the sphere: they are split, and the
    # queries whose own box is too full take the exhaustive path.  Measured:
    # 107 split items; 257 (FP32 filter) and 265 (FP64, whose split budget
    # is smaller) exhaustive queries.  The bounds hold that with a margin
    # for the few particles that change work item between builds.
    assert 0 < got[3]["split_items"] <= 130
    assert 0 < got[3]["brute_chunks"] <= 320


@pytest.mark.parametrize("prec", PRECS)
def test_row_paths(prec):
    """The main sweep's two ways to pass rows to pass 2: test words expanded
    by k_expand (items whose words take less room than their rows, among
    them items of more than 8192 row entries, expanded in windows) and rows
    in the scratch copied by k_place (items of few queries).  With 150
    neighbours a full item of 64 queries has about 9600 row entries and
    about 1200 candidates (inside the staging budget), while the short
    items at the end of leaves keep their rows.  Lists must equal the
    oracle's."""
    n = 60_000
    x, y, z, h = W.uniform_cube(n, 21, 150.0)
    log("row paths", prec)
    got = gpu_lists(x, y, z, h, prec, bucket_size=64)
    want = oracle.lists(x, y, z, h)
    assert_same_lists(got, want)
    st = got[3]
    log("row paths: items", st["n_chunks"], "words", st["word_items"], "wide",
        st["word_items_wide"], "split", st["split_items"])
    assert st["word_items_wide"] > 0
    assert st["word_items"] > st["word_items_wide"]
    assert st["n_chunks"] - st["word_items"] - st["split_items"] > 0


@pytest.mark.parametrize("prec", PRECS)
def test_split_paths(prec):
    """Work items whose candidates overflow shared memory: a few queries with
    a larger h make their item's box E too full (the item is re-searched in
    groups of 8 queries), and a few with a much larger h see more than a
    quarter of this small set (their item takes the exhaustive path).  Lists
    must still equal the oracle's."""
    n = 20_000
    x, y, z, h = W.uniform_cube(n, 7, 64.0)
    h = h.copy()
    h[::50] *= 1.6
    h[::997] *= 3.5
    log("split paths", prec)
    got = gpu_lists(x, y, z, h, prec, bucket_size=64)
    want = oracle.lists(x, y, z, h)
    assert_same_lists(got, want)
    st = got[3]
    assert st["split_items"] > 0
    assert 0 < st["brute_chunks"] <= 64 * len(h[::997])


@pytest.mark.parametrize("prec", PRECS)
def test_exhaustive_spans(prec):
    """Queries whose box covers most of a set larger than one span of the
    exhaustive count pass (9216 candidates): their rows are assembled from
    five spans counted and filled by separate workgroups, and must equal
    the oracle's."""
    n = 40_000
    x, y, z, h = W.uniform_cube(n, 11, 64.0)
    h = h.copy()
    big = np.arange(0, n, 200)
    h[big] = 0.45
    log("exhaustive spans", prec)
    got = gpu_lists(x, y, z, h, prec, bucket_size=64)
    check_csr_invariants(got[0], got[1], got[2], n)
    assert got[3]["brute_chunks"] >= len(big)
    rng = np.random.default_rng(3)
    rows = np.unique(np.concatenate([big, rng.integers(0, n, 300)]))
    assert_same_lists(got, oracle.lists(x, y, z, h, rows), rows)


@pytest.mark.parametrize("name,s,kw", [("U10k", 64, {}), ("P60k", 32, {}),
                                       ("P60k", 16, {"beta": 0.2}), ("L1M", 128, {}),
                                       ("P60k", 32, {"alpha": 0.25, "beta": 0.8}),
                                       ("P60k", 64, {"alpha": 1.0, "beta": 0.3}),
                                       ("U10k", 16, {"alpha": 0.125, "beta": 0.9})])
def test_tree_matches_algorithm1(name, s, kw):
    """Integer tree shape (leaf sizes, depths, members, b per cell) equals the
    oracle's recursive Algorithm 1, leaf by leaf in depth-first order."""
    from paper_1910_02639_amd import btree
    if name == "U10k":
        x, y, z, _ = W.uniform_cube(10_000, 0)
    elif name == "P60k":
        x, y, z, _ = W.plummer(60_000, 2)
    else:
        x, y, z, _ = W.lattice()
    log("tree", name, s, kw)
    ref = oracle.build_tree(x, y, z, s=s, **kw)
    dx, dy, dz = to_dev(x, y, z)
    with btree.BTree(dx, dy, dz, bucket_size=s, **kw) as t:
        st = t.stats()
        ex = t.export()
    assert st["n_leaves"] == ref.n_leaves
    assert st["n_internal"] == ref.n_internal
    assert st["depth"] == ref.depth
    assert st["rounds"] == ref.rounds
    assert st["b_hist"] == {b if b < 64 else 64: c for b, c in ref.b_hist.items()}
    assert np.array_equal(ex["leaf_cnt"], ref.leaf_cnt)
    assert np.array_equal(ex["leaf_depth"], ref.leaf_depth)
    off = ref.leaf_offsets()
    assert np.array_equal(ex["leaf_beg"], off[:-1])
    order = ex["order"]
    for l in range(ref.n_leaves):
        a = np.sort(order[off[l]:off[l + 1]])
        assert np.array_equal(a, ref.members[off[l]:off[l + 1]]), l


@pytest.mark.parametrize("prec", PRECS)
def test_parameter_grid_all_rows(prec):
    """The lists do not depend on s, beta or alpha (the tuner's axes, Eq. 4):
    every row of a 60k Plummer set against the oracle on a grid of them."""
    from paper_1910_02639_amd import btree
    import torch
    x, y, z, h = W.plummer(60_000, 23)
    dx, dy, dz, dh = to_dev(x, y, z, h)
    for s_ in (16, 64, 256):
        for beta in (0.3, 0.9):
            for alpha in (0.125, 1.0):
                log("grid", prec, s_, beta, alpha)
                with btree.BTree(dx, dy, dz, bucket_size=s_, beta=beta, alpha=alpha,
                                 precision=prec) as t:
                    c, o, nb = t.find(dh)
                    torch.cuda.synchronize()
                    assert_all_rows(x, y, z, h, c.cpu().numpy(), o.cpu().numpy(),
                                    nb.cpu().numpy(), "grid %d/%g/%g" % (s_, beta, alpha))


def _lattice_expected_counts(m=100):
    i = np.arange(m ** 3, dtype=np.int64)
    ix, iy, iz = i // (m * m), (i // m) % m, i % m
    cnt = np.zeros(m ** 3, dtype=np.int64)
    for a in range(-2, 3):
        for b in range(-2, 3):
            for c in range(-2, 3):
                if a * a + b * b + c * c <= 8:
                    ok = ((ix + a >= 0) & (ix + a < m) & (iy + b >= 0) & (iy + b < m) &
                          (iz + c >= 0) & (iz + c < m))
                    cnt += ok
    return cnt


@pytest.mark.parametrize("prec", PRECS)
def test_lattice_1m(prec):
    x, y, z, h = W.lattice()
    log("L1M", prec)
    c, o, nb, st = gpu_lists(x, y, z, h, prec, bucket_size=128)
    check_csr_invariants(c, o, nb, len(x))
    assert o[-1] == 90_205_144
    assert np.array_equal(c, _lattice_expected_counts())
    assert st["depth"] == 1 and st["n_leaves"] == 8000 and st["b_hist"] == {20: 1}
    assert_all_rows(x, y, z, h, c, o, nb, "L1M %s" % prec)
    # constant h: lists are symmetric
    r = np.repeat(np.arange(len(x), dtype=np.int64), c)
    fwd = r * len(x) + nb
    bwd = nb.astype(np.int64) * len(x) + r
    assert np.array_equal(np.sort(fwd), np.sort(bwd))


@pytest.mark.parametrize("prec", PRECS)
def test_plummer_8m_all_rows(prec):
    """P8M (8M-particle Plummer sphere), both arithmetic forms: every row
    equals the oracle's."""
    x, y, z, h = W.plummer(8_000_000, 0)
    log("P8M", prec)
    c, o, nb, st = gpu_lists(x, y, z, h, prec, bucket_size=128)
    log("P8M total", int(o[-1]), "exhaustive", st["brute_chunks"], "split", st["split_items"])
    assert_all_rows(x, y, z, h, c, o, nb, "P8M %s" % prec)
    assert st["brute_chunks"] == 0


def test_plummer_16m_precision_form():
    """The precision-form configuration: a 16M-particle Plummer sphere with
    the FP32 filter and FP64 band confirmation.  Every row equals the
    oracle's; the confirmed fraction is small but the band is exercised."""
    x, y, z, h = W.plummer(16_000_000, 0)
    log("P16M")
    c, o, nb, st = gpu_lists(x, y, z, h, "fp32", bucket_size=256, beta=0.8)
    log("P16M total", int(o[-1]), st["fp64_confirms"], st["pair_tests"])
    assert_all_rows(x, y, z, h, c, o, nb, "P16M")
    assert 0 < st["fp64_confirms"] < st["pair_tests"] * 1e-5


@pytest.mark.parametrize("prec", PRECS)
def test_edge_cases(prec):
    rng = np.random.default_rng(17)
    # coincident particles beyond the bucket size (depth guard), plus others
    x = np.concatenate([np.full(300, 0.25), rng.random(700)])
    y = np.concatenate([np.full(300, 0.5), rng.random(700)])
    z = np.concatenate([np.full(300, 0.75), rng.random(700)])
    h = np.full(1000, 0.02)
    got = gpu_lists(x, y, z, h, prec, bucket_size=16, max_depth=12)
    assert_same_lists(got, oracle.lists(x, y, z, h))
    assert got[3]["oversized"] >= 1
    # leaves of 700 and 1500 coincident particles at the depth guard: the
    # workgroup sort (513..1024 particles) and the order-keeping copy above
    for m in (700, 1500):
        x = np.concatenate([np.full(m, 0.3), rng.random(500)])
        y = np.concatenate([np.full(m, 0.6), rng.random(500)])
        z = np.concatenate([np.full(m, 0.2), rng.random(500)])
        h = np.full(m + 500, 0.02)
        got = gpu_lists(x, y, z, h, prec, bucket_size=16, max_depth=6)
        assert_same_lists(got, oracle.lists(x, y, z, h))
        assert got[3]["max_leaf"] >= m
    # a plane (zero extent along z) and a line
    x, y = rng.random((2, 3000))
    z = np.zeros(3000)
    h = np.full(3000, 0.03)
    assert_same_lists(gpu_lists(x, y, z, h, prec, bucket_size=32),
                      oracle.lists(x, y, z, h))
    y = np.zeros(3000)
    assert_same_lists(gpu_lists(x, y, z, h, prec, bucket_size=32),
                      oracle.lists(x, y, z, h))
    # far from the origin, negative coordinates
    x, y, z, h = W.uniform_cube(5000, 3, 64.0)
    x = x * 1e-3 - 1e6
    y = y * 1e-3 + 3e5
    z = z * 1e-3
    h = h * 1e-3
    assert_same_lists(gpu_lists(x, y, z, h, prec), oracle.lists(x, y, z, h))
    # scales where FP32 squares overflow (2^70) or flush to zero (2^-70):
    # the FP32 filter must hand such items to FP64 arithmetic
    x, y, z, h = W.uniform_cube(3000, 5, 64.0)
    for scale in (2.0 ** 70, 2.0 ** -70):
        xs, ys, zs, hs = x * scale, y * scale, z * scale, h * scale
        assert_same_lists(gpu_lists(xs, ys, zs, hs, prec), oracle.lists(xs, ys, zs, hs))
    # all zero h: every row empty
    x, y, z, h = W.uniform_cube(3000, 4, 64.0)
    got = gpu_lists(x, y, z, np.zeros(3000), prec)
    assert got[0].sum() == 0
    # radius above the diagonal: every row is 0..n-1 (exhaustive path)
    got = gpu_lists(x[:2500], y[:2500], z[:2500], np.full(2500, 5.0), prec)
    assert np.all(got[0] == 2500)
    assert np.array_equal(got[2].reshape(2500, 2500), np.tile(np.arange(2500), (2500, 1)))


@pytest.mark.parametrize("prec", PRECS)
def test_band_pairs_exact(prec):
    """Pairs placed on, just inside and just outside 2h_i (relative steps of
    a few FP32 ulps) go through the FP64 confirmation and still match."""
    rng = np.random.default_rng(23)
    n0 = 400
    cx, cy, cz = rng.random((3, n0)) * 10.0
    hq = rng.uniform(0.01, 0.1, n0)
    xs, ys, zs, hs = [cx], [cy], [cz], [hq]
    for k in (-3, -1, 0, 1, 3):
        d = rng.normal(size=(3, n0))
        d /= np.linalg.norm(d, axis=0)
        R = 2.0 * hq * (1.0 + k * 2.0 ** -24)
        xs.append(cx + R * d[0]); ys.append(cy + R * d[1]); zs.append(cz + R * d[2])
        hs.append(np.full(n0, 0.001))
    # exact ties along an axis: x_j = x_i + 2h_i with representable values
    tx = np.arange(n0, dtype=np.float64) * 4.0
    xs.append(tx); ys.append(np.full(n0, 50.0)); zs.append(np.zeros(n0)); hs.append(np.full(n0, 0.5))
    xs.append(tx + 1.0); ys.append(np.full(n0, 50.0)); zs.append(np.zeros(n0)); hs.append(np.full(n0, 0.25))
    x, y, z, h = (np.concatenate(v) for v in (xs, ys, zs, hs))
    got = gpu_lists(x, y, z, h, prec, bucket_size=32)
    assert_same_lists(got, oracle.lists(x, y, z, h))
    if prec == "fp32":
        assert got[3]["fp64_confirms"] > 0


def test_empty_and_invalid():
    import torch
    from paper_1910_02639_amd import btree
    e = torch.empty(0, dtype=torch.float64, device="cuda:0")
    with btree.BTree(e, e, e) as t:
        c, o, nb = t.find(e)
        assert o.cpu().tolist() == [0] and nb.numel() == 0
    x, y, z, h = W.uniform_cube(2000, 5, 64.0)
    dx, dy, dz, dh = to_dev(x, y, z, h)
    bad = dh.clone()
    bad[17] = float("nan")
    with btree.BTree(dx, dy, dz) as t:
        counts = torch.full((2000,), -7, dtype=torch.int32, device="cuda:0")
        offs = torch.full((2001,), -7, dtype=torch.int64, device="cuda:0")
        with pytest.raises(btree.BTreeError) as ei:
            t.count(bad, counts, offs)
        assert ei.value.status == btree.BTREE_EINVAL
        assert int((counts != -7).sum()) == 0 and int((offs != -7).sum()) == 0
        neg = dh.clone()
        neg[3] = -1.0
        with pytest.raises(btree.BTreeError):
            t.count(neg)
        # a valid call still works after the failures
        c, o, tot = t.count(dh)
        small = torch.empty(max(tot - 1, 0), dtype=torch.int32, device="cuda:0")
        with pytest.raises(btree.BTreeError) as ei:
            t.fill(dh, c, o, small)
        assert ei.value.status == btree.BTREE_EOVERFLOW
    xb = dx.clone()
    xb[5] = float("inf")
    with pytest.raises(btree.BTreeError) as ei:
        btree.BTree(xb, dy, dz)
    assert ei.value.status == btree.BTREE_EINVAL


@pytest.mark.parametrize("prec", PRECS)
def test_deterministic(prec):
    x, y, z, h = W.plummer(200_000, 8)
    a = gpu_lists(x, y, z, h, prec, bucket_size=64)
    b = gpu_lists(x, y, z, h, prec, bucket_size=64)
    for u, v in zip(a[:3], b[:3]):
        assert np.array_equal(u, v)
    # parameter independence of the result
    c = gpu_lists(x, y, z, h, "fp64" if prec == "fp32" else "fp32", bucket_size=16, beta=0.3)
    for u, v in zip(a[:3], c[:3]):
        assert np.array_equal(u, v)


@pytest.mark.parametrize("prec", PRECS)
def test_rebuild_deeper_than_before(prec):
    """A rebuild queues the previous tree's level count plus one with no host
    read between levels; a tree that needs more levels is built again level
    by level.  A one-level tree (uniform set, s = 512), then a Plummer set
    whose tree is deeper: same lists and tree depth as a fresh build."""
    from paper_1910_02639_amd import btree
    import torch
    xu, yu, zu, hu = W.uniform_cube(20_000, 13, 64.0)
    xp, yp, zp, hp = W.plummer(60_000, 14)
    U = to_dev(xu, yu, zu, hu)
    Pd = to_dev(xp, yp, zp, hp)
    with btree.BTree(Pd[0], Pd[1], Pd[2], bucket_size=512, precision=prec) as fresh:
        depth_p = fresh.stats()["depth"]
    with btree.BTree(U[0], U[1], U[2], bucket_size=512, precision=prec) as t:
        assert t.stats()["depth"] == 1
        assert depth_p >= 3  # more than the one level queued beyond the last tree's
        t.rebuild(Pd[0], Pd[1], Pd[2])
        assert t.stats()["depth"] == depth_p
        c, o, nb = t.find(Pd[3])
        torch.cuda.synchronize()
        assert_same_lists((c.cpu().numpy(), o.cpu().numpy(), nb.cpu().numpy()),
                          oracle.lists(xp, yp, zp, hp))
        t.rebuild(U[0], U[1], U[2])
        assert t.stats()["depth"] == 1
        c, o, nb = t.find(U[3])
        torch.cuda.synchronize()
        assert_same_lists((c.cpu().numpy(), o.cpu().numpy(), nb.cpu().numpy()),
                          oracle.lists(xu, yu, zu, hu))


@pytest.mark.parametrize("prec", PRECS)
def test_rebuild_reuses_handle(prec):
    """btree_rebuild over a different set (and size) gives that set's lists;
    phase timers accumulate across rebuilds."""
    from paper_1910_02639_amd import btree
    import torch
    xa, ya, za, ha = W.plummer(50_000, 11)
    xb, yb, zb, hb = W.uniform_cube(20_000, 12, 64.0)
    A = to_dev(xa, ya, za, ha)
    B = to_dev(xb, yb, zb, hb)
    with btree.BTree(A[0], A[1], A[2], bucket_size=32, precision=prec, timing=True) as t:
        c, o, nb = t.find(A[3])
        assert_same_lists((c.cpu().numpy(), o.cpu().numpy(), nb.cpu().numpy()),
                          oracle.lists(xa, ya, za, ha))
        t.rebuild(B[0], B[1], B[2])
        c, o, nb = t.find(B[3])
        assert_same_lists((c.cpu().numpy(), o.cpu().numpy(), nb.cpu().numpy()),
                          oracle.lists(xb, yb, zb, hb))
        t.rebuild(A[0], A[1], A[2])
        c, o, nb = t.find(A[3])
        torch.cuda.synchronize()
        assert_same_lists((c.cpu().numpy(), o.cpu().numpy(), nb.cpu().numpy()),
                          oracle.lists(xa, ya, za, ha))
        st = t.stats()
        assert st["phase_calls"]["build"] == 3 and st["phase_ms"]["build"] > 0
        # a pass 1 whose walk lists or rows outgrew the handle's pools runs
        # the sweep again after growing them (never more than twice)
        assert 3 <= st["phase_calls"]["sweep_kernel"] <= 9
        assert st["phase_calls"]["place_kernel"] == 3
