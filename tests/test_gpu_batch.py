"""GPU parity of the batched form (btree_batch_*): every set of a batch
against the FP64 oracle run on that set alone, element by element, and the
captured graph replayed with eager work and new data between replays."""
import numpy as np
import pytest

import oracle
from paper_1910_02639_amd import workloads as W
from tests.helpers import assert_all_rows, log, to_dev

pytestmark = pytest.mark.gpu

PRECS = ["fp32", "fp64"]


@pytest.fixture(scope="module", autouse=True)
def _setup():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    oracle.build(force=False)


def _mixed_sets(sizes, seed):
    """Sets of the given sizes: cube, Plummer and Gaussian blobs in turn,
    each with its own h rule; some h = 0."""
    out = []
    for k, n in enumerate(sizes):
        if n == 0:
            e = np.zeros(0)
            out.append((e, e, e, e))
            continue
        kind = k % 3
        if kind == 0:
            x, y, z, h = W.uniform_cube(n, seed + k, 40.0)
        elif kind == 1:
            x, y, z, h = W.plummer(n, seed + k, 60.0)
        else:
            rng = np.random.default_rng(seed + k)
            x, y, z = rng.normal(size=(3, n)) * 0.3 + k
            h = rng.uniform(0.02, 0.2, n)
            h[::5] = 0.0
        out.append((x, y, z, h))
    return out


def _concat(sets):
    return [np.concatenate([s[c] for s in sets]) for c in range(4)]


def _check_batch(sets, counts, offsets, nbrs, totals):
    """Each set's block of the batch CSR equals the oracle on that set."""
    beg = 0
    for k, (x, y, z, h) in enumerate(sets):
        n = len(x)
        if n == 0:
            assert totals[k] == 0
            continue
        wc, wo, wn = oracle.lists(x, y, z, h)
        gc = counts[beg:beg + n].astype(np.int64)
        go = offsets[beg:beg + n + 1]
        assert np.array_equal(gc, wc), "set %d counts differ" % k
        assert np.array_equal(go - go[0], wo), "set %d offsets differ" % k
        assert np.array_equal(nbrs[go[0]:go[-1]], wn), "set %d lists differ" % k
        assert totals[k] == wo[-1]
        beg += n


def _host(*ts):
    return [t.cpu().numpy() for t in ts]


@pytest.mark.parametrize("prec", PRECS)
def test_batch_mixed_sets(prec):
    """Uneven sets (empty, one particle, a single leaf, several levels) with
    per-set parameters, in one graph launch."""
    from paper_1910_02639_amd import btree
    sizes = [0, 1, 500, 3000, 20000, 64, 0, 7000]
    sets = _mixed_sets(sizes, 11)
    prm = [dict(bucket_size=s, beta=b) for s, b in
           zip([64, 8, 32, 16, 128, 64, 64, 24], [0.5, 0.5, 0.3, 0.5, 0.5, 0.8, 0.5, 0.5])]
    log("batch mixed", prec)
    x, y, z, h = to_dev(*_concat(sets))
    with btree.Batch(sizes, prm, precision=prec) as B:
        c, o, nb, totals = B.find(x, y, z, h)
        _check_batch(sets, *_host(c, o, nb), totals)
        st = B.stats()
        assert st["n"] == sum(sizes)
        assert st["total"] == int(totals.sum())


@pytest.mark.parametrize("prec", PRECS)
def test_graph_replays_with_new_data(prec):
    """The same graph replayed three times: between replays the program does
    its own eager GPU work and writes new particles into the same buffers;
    every replay must match the oracle on the data it saw."""
    import torch
    from paper_1910_02639_amd import btree
    sizes = [4000, 900, 12000]
    cap = 16_000_000
    xs = [to_dev(*_concat(_mixed_sets(sizes, s))) for s in (21, 22, 23)]
    x, y, z, h = [t.clone() for t in xs[0]]
    n = sum(sizes)
    counts = torch.empty(n, dtype=torch.int32, device="cuda:0")
    offsets = torch.empty(n + 1, dtype=torch.int64, device="cuda:0")
    nbrs = torch.empty(cap, dtype=torch.int32, device="cuda:0")
    with btree.Batch(sizes, precision=prec, bucket_size=32, timing=True) as B:
        for r, seed in enumerate((21, 22, 23)):
            log("replay", r, prec)
            for dst, src in zip((x, y, z, h), xs[r]):
                dst.copy_(src)
            # unrelated eager work on the same stream, then a full sync
            junk = torch.randn(1 << 20, device="cuda:0").sum()
            torch.cuda.synchronize()
            totals, total = B.run(x, y, z, h, counts, offsets, nbrs)
            _check_batch(_mixed_sets(sizes, seed), *_host(counts, offsets, nbrs[:total]), totals)
            assert float(junk) == float(junk)
        st = B.stats()
        assert st["graph_launches"] >= 3
        # one recording unless new data outgrew a pool
        assert st["graph_captures"] <= 3
        # HIP events between graph segments time every phase of every replay
        for k in ("build", "sweep_kernel", "place_kernel", "pass1", "pass2"):
            assert st["phase_calls"][k] == st["graph_launches"], k
            assert st["phase_ms"][k] > 0.0, k


def test_pool_regrow_and_recapture():
    """A replay whose data needs more tree levels than the recorded graph
    holds is detected on the device, the handle grows and records again,
    and the result is still exact."""
    import torch
    from paper_1910_02639_amd import btree
    n = 6000
    x0, y0, z0, h0 = W.uniform_cube(n, 3, 40.0)
    rng = np.random.default_rng(4)
    # clustered: nested blobs need several levels at s = 16
    x1 = np.concatenate([rng.normal(size=n // 2) * 1e-3, rng.random(n - n // 2)])
    y1 = np.concatenate([rng.normal(size=n // 2) * 1e-3, rng.random(n - n // 2)])
    z1 = np.concatenate([rng.normal(size=n // 2) * 1e-3, rng.random(n - n // 2)])
    h1 = np.full(n, 2e-4)
    x, y, z, h = to_dev(x0, y0, z0, h0)
    counts = torch.empty(n, dtype=torch.int32, device="cuda:0")
    offsets = torch.empty(n + 1, dtype=torch.int64, device="cuda:0")
    nbrs = torch.empty(2_000_000, dtype=torch.int32, device="cuda:0")
    with btree.Batch([n], bucket_size=16) as B:
        totals, total = B.run(x, y, z, h, counts, offsets, nbrs)
        _check_batch([(x0, y0, z0, h0)], *_host(counts, offsets, nbrs[:total]), totals)
        caps0 = B.stats()["graph_captures"]
        for dst, src in zip((x, y, z, h), to_dev(x1, y1, z1, h1)):
            dst.copy_(src)
        log("regrow")
        totals, total = B.run(x, y, z, h, counts, offsets, nbrs)
        _check_batch([(x1, y1, z1, h1)], *_host(counts, offsets, nbrs[:total]), totals)
        st = B.stats()
        assert st["graph_captures"] > caps0
        assert st["depth"] >= 3


def test_batch_capacity_overflow():
    import torch
    from paper_1910_02639_amd import btree
    sizes = [3000, 2000]
    sets = _mixed_sets(sizes, 31)
    x, y, z, h = to_dev(*_concat(sets))
    n = sum(sizes)
    counts = torch.empty(n, dtype=torch.int32, device="cuda:0")
    offsets = torch.empty(n + 1, dtype=torch.int64, device="cuda:0")
    small = torch.full((100,), -7, dtype=torch.int32, device="cuda:0")
    with btree.Batch(sizes) as B:
        with pytest.raises(btree.BTreeError) as e:
            B.run(x, y, z, h, counts, offsets, small)
        assert e.value.status == btree.BTREE_EOVERFLOW
        want = [oracle.lists(*s)[1][-1] for s in sets]
        assert list(B.last_totals) == want
        assert (small.cpu().numpy() == -7).all()  # untouched
        big = torch.empty(B.last_total, dtype=torch.int32, device="cuda:0")
        totals, total = B.run(x, y, z, h, counts, offsets, big)
        _check_batch(sets, *_host(counts, offsets, big), totals)


def test_batch_bad_h_rejected():
    import torch
    from paper_1910_02639_amd import btree
    sizes = [500, 500]
    sets = _mixed_sets(sizes, 41)
    xs, ys, zs, hs = _concat(sets)
    hs[700] = -1.0
    x, y, z, h = to_dev(xs, ys, zs, hs)
    counts = torch.full((1000,), -3, dtype=torch.int32, device="cuda:0")
    offsets = torch.empty(1001, dtype=torch.int64, device="cuda:0")
    nbrs = torch.empty(10, dtype=torch.int32, device="cuda:0")
    with btree.Batch(sizes) as B:
        with pytest.raises(btree.BTreeError) as e:
            B.run(x, y, z, h, counts, offsets, nbrs)
        assert e.value.status == btree.BTREE_EINVAL
        assert (counts.cpu().numpy() == -3).all()


def test_batch_all_empty():
    import torch
    from paper_1910_02639_amd import btree
    e = torch.zeros(0, dtype=torch.float64, device="cuda:0")
    counts = torch.zeros(1, dtype=torch.int32, device="cuda:0")
    offsets = torch.full((1,), 5, dtype=torch.int64, device="cuda:0")
    nbrs = torch.zeros(1, dtype=torch.int32, device="cuda:0")
    with btree.Batch([0, 0, 0]) as B:
        totals, total = B.run(e, e, e, e, counts, offsets, nbrs)
        assert total == 0 and list(totals) == [0, 0, 0]
        assert int(offsets[0]) == 0


@pytest.mark.parametrize("prec", PRECS)
def test_batch64_shape_matches_single_trees(prec):
    """A reduced Batch64 (16 sets, sizes log-uniform in [10^3.5, 10^4.6]):
    each set's lists equal btree_build + btree_find_neighbors on the set
    alone, and sampled rows equal the oracle."""
    import torch
    from paper_1910_02639_amd import btree
    sets = W.batch(16, 0, 3.5, 4.6)
    sizes = [len(s[0]) for s in sets]
    log("batch16", prec, sum(sizes))
    x, y, z, h = to_dev(*_concat(sets))
    with btree.Batch(sizes, precision=prec, bucket_size=64) as B:
        c, o, nb, totals = B.find(x, y, z, h)
        c, o, nb = _host(c, o, nb)
    beg = 0
    rng = np.random.default_rng(5)
    for k, (xs, ys, zs, hs) in enumerate(sets):
        n = len(xs)
        dx, dy, dz, dh = to_dev(xs, ys, zs, hs)
        with btree.BTree(dx, dy, dz, bucket_size=64, precision=prec) as t:
            sc, so, sn = t.find(dh)
            torch.cuda.synchronize()
            sc, so, sn = _host(sc, so, sn)
        go = o[beg:beg + n + 1]
        assert np.array_equal(c[beg:beg + n], sc)
        assert np.array_equal(go - go[0], so)
        assert np.array_equal(nb[go[0]:go[-1]], sn)
        rows = rng.choice(n, 20, replace=False)
        for i in rows:
            r = oracle.row(xs, ys, zs, hs, int(i))
            assert np.array_equal(sn[so[i]:so[i + 1]], r)
        beg += n


def test_batch64_full_size_all_rows():
    """The full Batch64 workload (64 sets, 13.5 M particles) in the form the
    benchmark times: tuned parameters per set, FP32 filter, the captured
    graph replayed.  Replays equal the first run, and every row of every set
    equals the oracle's.  The FP64 batched form (its own tuned parameters)
    gives the same bytes."""
    import torch
    from paper_1910_02639_amd import autotune, btree
    sets = W.batch(64, 0)
    sizes = [len(s[0]) for s in sets]
    n = int(sum(sizes))
    log("Batch64 full", n)
    dx, dy, dz, dh = to_dev(*_concat(sets))
    offs = np.zeros(len(sizes) + 1, dtype=np.int64)
    np.cumsum(sizes, out=offs[1:])
    tuner = autotune.Tuner(autotune.CACHE, tune_missing=False)
    views = [(dx[offs[k]:offs[k + 1]], dy[offs[k]:offs[k + 1]], dz[offs[k]:offs[k + 1]],
              dh[offs[k]:offs[k + 1]]) for k in range(len(sizes))]
    prm = [tuner.params_for(*v, "fp32") for v in views]
    with btree.Batch(sizes, prm, precision="fp32") as B:
        c0, o0, nb0, totals = B.find(dx, dy, dz, dh)
        total = int(totals.sum())
        counts = torch.empty(n, dtype=torch.int32, device="cuda:0")
        offsets = torch.empty(n + 1, dtype=torch.int64, device="cuda:0")
        nbrs = torch.empty(total, dtype=torch.int32, device="cuda:0")
        for rep in range(2):
            nbrs.fill_(-1)
            t2, tot2 = B.run(dx, dy, dz, dh, counts, offsets, nbrs)
            torch.cuda.synchronize()
            assert tot2 == total and list(t2) == list(totals)
            assert torch.equal(counts, c0) and torch.equal(offsets, o0)
            assert torch.equal(nbrs, nb0), "replay %d differs from the first run" % rep
    del counts, offsets, nbrs
    log("Batch64 total", total, "fp64 batched form")
    prm64 = [tuner.params_for(*v, "fp64") for v in views]
    with btree.Batch(sizes, prm64, precision="fp64") as B:
        c1, o1, nb1, totals1 = B.find(dx, dy, dz, dh)
        torch.cuda.synchronize()
    assert list(totals1) == list(totals)
    assert torch.equal(c1, c0) and torch.equal(o1, o0) and torch.equal(nb1, nb0)
    del c1, o1, nb1
    c, oh, nbh = _host(c0, o0, nb0)
    assert int(oh[0]) == 0 and int(oh[-1]) == total == nbh.shape[0]
    for k, (xs, ys, zs, hs) in enumerate(sets):
        b, e = int(offs[k]), int(offs[k + 1])
        so = oh[b:e + 1] - oh[b]
        assert_all_rows(xs, ys, zs, hs, c[b:e], so, nbh[int(oh[b]):int(oh[e])],
                        "Batch64 set %d" % k)
    log("Batch64 every row equal")


def test_tuner_picks_a_candidate_and_results_do_not_depend_on_it():
    """btree_tune times every candidate (device time of the recorded graph)
    and returns the fastest; lists with any candidate equal the oracle's."""
    from paper_1910_02639_amd import autotune, btree
    x, y, z, h = W.uniform_cube(8000, 9, 40.0)
    dx, dy, dz, dh = to_dev(x, y, z, h)
    sp = autotune.space(buckets=[16, 64], betas=[0.5, 0.8], repeats=2, alphas=[0.25, 1.0])
    r = autotune.tune(dx, dy, dz, dh, "fp32", sp)
    assert r["bucket_size"] in (16, 64) and r["beta"] in (0.5, 0.8) and r["alpha"] in (0.25, 1.0)
    assert len(r["table"]) == 8
    assert r["ms"] > 0 and all(v > 0 for v in r["table"].values())
    assert r["ms"] == min(r["table"].values())
    assert r["table"]["%d/%g/%g" % (r["bucket_size"], r["beta"], r["alpha"])] == r["ms"]
    want = oracle.lists(x, y, z, h)
    for s, a in ((16, 0.25), (64, 1.0)):
        with btree.Batch([len(x)], bucket_size=s, beta=r["beta"], alpha=a) as B:
            c, o, nb, totals = B.find(dx, dy, dz, dh)
            _check_batch([(x, y, z, h)], *_host(c, o, nb), totals)
    assert want[1][-1] == totals[0]


def test_batch_handles_release_memory():
    """Creating, running and closing batch handles returns their device
    memory: free memory after the third cycle is within 256 MiB of the
    first (a handle of this size holds about 1 GiB)."""
    import torch
    from paper_1910_02639_amd import btree
    x, y, z, h = W.plummer(2_000_000, 4, 100.0)
    dx, dy, dz, dh = to_dev(x, y, z, h)
    log("batch memory release")
    free = []
    for _ in range(3):
        B = btree.Batch([len(x)], [dict(bucket_size=64)])
        c, o, nb, _ = B.find(dx, dy, dz, dh)
        del c, o, nb
        B.close()
        del B
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
        free.append(torch.cuda.mem_get_info()[0])
    assert free[2] >= free[0] - 256 * 2 ** 20, free
