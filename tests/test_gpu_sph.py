"""GPU parity of the SPH uses of the search, through the C ABI:

* btree_density (the fused consumer: density sums inside the search, no
  lists) against the oracle's density over its rows.  Counts must be equal.
  Each term m_j w(r_ij / h_i) is the same IEEE operations in the same order
  on both sides, so densities differ only by the order of the additions: for
  k positive terms, two orders differ by at most 2 (k - 1) u times the sum
  (u = 2^-53), the tolerance used here.
* btree_adapt_h against the oracle's adaptation: counts are exact integers
  and each update is the same single-rounded operations, so h must be equal
  bit for bit, with the same counts and the same number of rounds.
"""
import numpy as np
import pytest

import oracle
from paper_1910_02639_amd import workloads as W
from tests.helpers import log, to_dev

pytestmark = pytest.mark.gpu

PRECS = ["fp32", "fp64"]
U = 2.0 ** -53


@pytest.fixture(scope="module", autouse=True)
def _setup():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    oracle.build(force=False)


def _gpu_density(x, y, z, h, prec, mass=None, **kw):
    import torch
    from paper_1910_02639_amd import btree
    dx, dy, dz, dh = to_dev(x, y, z, h)
    dm = to_dev(mass)[0] if mass is not None else None
    with btree.BTree(dx, dy, dz, precision=prec, **kw) as t:
        rho, c = t.density(dh, dm)
        torch.cuda.synchronize()
        st = t.stats()
    return rho.cpu().numpy(), c.cpu().numpy().astype(np.int64), st


def _check_density(got_rho, got_c, want_rho, want_c, what):
    assert np.array_equal(got_c, want_c), "%s: counts differ at %s" % (
        what, np.nonzero(got_c != want_c)[0][:10])
    tol = 2.0 * np.maximum(want_c - 1, 0) * U * np.abs(want_rho)
    bad = np.nonzero(np.abs(got_rho - want_rho) > tol)[0]
    assert bad.size == 0, "%s: densities differ at %s (%s vs %s)" % (
        what, bad[:5], got_rho[bad[:5]], want_rho[bad[:5]])


def _density_cases():
    rng = np.random.default_rng(51)
    x, y, z, h = W.uniform_cube(20_000, 7, 64.0)
    h = h.copy()
    h[::50] *= 1.6
    h[::997] *= 3.5      # split levels and the exhaustive path
    return [("U10k", W.uniform_cube(10_000, 0, 64.0), 64, None),
            ("P30k", W.plummer(30_000, 5), 32, rng.uniform(0.5, 2.0, 30_000)),
            ("split paths", (x, y, z, h), 64, None)]


@pytest.mark.parametrize("prec", PRECS)
def test_density_equals_oracle(prec):
    for name, (x, y, z, h), s, m in _density_cases():
        log("density", name, prec)
        rho, c, st = _gpu_density(x, y, z, h, prec, mass=m, bucket_size=s)
        want_rho, want_c = oracle.density(x, y, z, h, mass=m)
        _check_density(rho, c, want_rho, want_c, name)
        if name == "split paths":
            assert st["split_items"] > 0 and st["brute_chunks"] > 0


@pytest.mark.parametrize("prec", PRECS)
def test_density_options(prec):
    x, y, z, h = W.plummer(20_000, 8)
    for kw in (dict(exclude_self=True), dict(octree=True, bucket_size=16)):
        log("density", kw, prec)
        rho, c, _ = _gpu_density(x, y, z, h, prec, **kw)
        want_rho, want_c = oracle.density(x, y, z, h, exclude_self=kw.get("exclude_self", False))
        _check_density(rho, c, want_rho, want_c, str(kw))


_DENS_P8M = {}


@pytest.mark.parametrize("prec", PRECS)
def test_density_p8m_all_particles(prec):
    """P8M (8M-particle Plummer sphere, masses drawn from [0.5, 2]) at the
    parameters the timing runs use: every particle's count equals the
    oracle's and every density lies within the summation-order bound."""
    x, y, z, h = W.plummer(8_000_000, 0)
    m = np.random.default_rng(52).uniform(0.5, 2.0, len(x))
    log("density P8M", prec)
    rho, c, st = _gpu_density(x, y, z, h, prec, mass=m, bucket_size=256, beta=0.8, alpha=0.25)
    if not _DENS_P8M:
        log("density P8M oracle")
        _DENS_P8M["want"] = oracle.density(x, y, z, h, mass=m)
    want_rho, want_c = _DENS_P8M["want"]
    log("density P8M split items", st["split_items"], "exhaustive", st["brute_chunks"])
    _check_density(rho, c, want_rho, want_c, "P8M " + prec)


def test_density_matches_lists_and_repeats():
    """Counts of the fused pass equal the lists' counts; two runs give the
    same bytes; a zero-h particle has density 0."""
    import torch
    from paper_1910_02639_amd import btree
    x, y, z, h = W.uniform_cube(15_000, 9, 64.0)
    h = h.copy()
    h[::13] = 0.0
    dx, dy, dz, dh = to_dev(x, y, z, h)
    with btree.BTree(dx, dy, dz, bucket_size=48) as t:
        r1, c1 = t.density(dh)
        r2, c2 = t.density(dh)
        cl, ol, nb = t.find(dh)
        torch.cuda.synchronize()
    assert torch.equal(r1, r2) and torch.equal(c1, c2) and torch.equal(c1, cl)
    assert float(r1[::13].abs().max()) == 0.0


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("gen,T,tol,scale", [("cube", 64, 2, 0.5), ("cube", 100, 0, 1.3),
                                            ("plummer", 100, 3, 0.7), ("lattice", 100, 0, 0.5)])
def test_adapt_h_equals_oracle(prec, gen, T, tol, scale):
    import torch
    from paper_1910_02639_amd import btree
    if gen == "cube":
        x, y, z, h = W.uniform_cube(30_000, 3, 64.0)
    elif gen == "plummer":
        x, y, z, h = W.plummer(30_000, 4)
    else:
        x, y, z, h = W.lattice(30, 0)
    h0 = h * scale
    log("adapt_h", gen, T, tol, scale, prec)
    want_h, want_c, want_it = oracle.adapt_h(x, y, z, h0, T, tol, 60)
    dx, dy, dz, dh = to_dev(x, y, z, h0)
    with btree.BTree(dx, dy, dz, bucket_size=64, precision=prec) as t:
        c, it = t.adapt_h(dh, T, tol, 60)
        torch.cuda.synchronize()
    assert it == want_it
    assert np.array_equal(c.cpu().numpy().astype(np.int64), want_c)
    assert np.array_equal(dh.cpu().numpy(), want_h), "h differs from the oracle's"


_ADAPT_1M = {}


@pytest.mark.parametrize("prec", PRECS)
def test_adapt_h_plummer_1m(prec):
    """A 1M-particle Plummer sphere from 0.7 h to 100 +- 3 neighbours: the
    same rounds, counts and h, bit for bit, as the oracle's adaptation."""
    import torch
    from paper_1910_02639_amd import btree
    x, y, z, h = W.plummer(1_000_000, 3)
    h0 = h * 0.7
    if not _ADAPT_1M:
        log("adapt_h 1M oracle")
        _ADAPT_1M["want"] = oracle.adapt_h(x, y, z, h0, 100.0, 3.0, 60)
    want_h, want_c, want_it = _ADAPT_1M["want"]
    log("adapt_h 1M", prec, "rounds", want_it)
    dx, dy, dz, dh = to_dev(x, y, z, h0)
    with btree.BTree(dx, dy, dz, bucket_size=128, precision=prec) as t:
        c, it = t.adapt_h(dh, 100.0, 3.0, 60)
        torch.cuda.synchronize()
    assert it == want_it
    assert np.array_equal(c.cpu().numpy().astype(np.int64), want_c)
    assert np.array_equal(dh.cpu().numpy(), want_h), "h differs from the oracle's"


def test_adapt_h_zero_rounds_and_errors():
    import torch
    from paper_1910_02639_amd import btree
    x, y, z, h = W.uniform_cube(5_000, 6, 64.0)
    dx, dy, dz, dh = to_dev(x, y, z, h)
    with btree.BTree(dx, dy, dz) as t:
        _, c0 = t.density(dh)
        c, it = t.adapt_h(dh, 64, 1000, 10)  # every count within the tolerance
        assert it == 0 and torch.equal(c, c0)
        for bad in (dict(target=0.0), dict(target=float("nan")), dict(target=64, tol=-1.0),
                    dict(target=64, max_iter=1001)):
            kw = dict(tol=0.0, max_iter=10)
            kw.update(bad)
            with pytest.raises(btree.BTreeError) as ei:
                t.adapt_h(dh, **kw)
            assert ei.value.status == btree.BTREE_EINVAL
