"""Pins of the oracle's cell-list evaluation and of its octree option.

The cell list computes the same lists as the brute-force definition (every
j tested with the FP64 predicate), only faster; it is what lets the GPU
tests compare every row at millions of particles.  It is pinned here by byte
equality with the brute force on many inputs, including degenerate ones,
and by the closed form of the jittered lattice on every row of L1M.  Planted
mistakes (compiled from a modified copy of the oracle source, on the CPU)
must each fail one of these pins.

The octree option of the oracle's BuildTree (b = 2 at every split) is pinned
by a hand-built example and by its agreement with Algorithm 1 run with a
ratio threshold no sub-cell distribution can satisfy (beta < 0 halves b down
to 2 at every cell).
"""
import ctypes
import os
import subprocess

import numpy as np
import pytest

from paper_1910_02639_amd import workloads as W

HERE = os.path.dirname(os.path.abspath(__file__))
ORACLE_C = os.path.join(os.path.dirname(HERE), "oracle", "oracle.c")


def _brute_vs_cells(oracle_mod, x, y, z, h):
    a = oracle_mod.lists(x, y, z, h)
    b = oracle_mod.cell_lists(x, y, z, h)
    assert np.array_equal(a[0], b[0]), "counts differ"
    assert np.array_equal(a[1], b[1]), "offsets differ"
    assert np.array_equal(a[2], b[2]), "lists differ"
    k, bad = oracle_mod.cell_check(x, y, z, h, a[0].astype(np.int32), a[1], a[2])
    assert k == 0, bad
    return a


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_cells_equal_brute_uniform_10k(oracle_mod, seed):
    x, y, z, h = W.uniform_cube(10_000, seed, 64.0)
    _brute_vs_cells(oracle_mod, x, y, z, h)


@pytest.mark.parametrize("n,seed", [(30_000, 5), (60_000, 2)])
def test_cells_equal_brute_plummer(oracle_mod, n, seed):
    # h spans about a factor 40 here: several cell levels are used.
    x, y, z, h = W.plummer(n, seed)
    _brute_vs_cells(oracle_mod, x, y, z, h)


def _edge_sets():
    rng = np.random.default_rng(77)
    out = {}
    x, y, z, h = W.uniform_cube(3000, 3, 64.0)
    out["h_zero"] = (x, y, z, np.zeros_like(h))
    out["h_mixed_zero"] = (x, y, z, np.where(np.arange(3000) % 3 == 0, 0.0, h))
    out["radius_above_diagonal"] = (x, y, z, np.full(3000, 5.0))
    out["radius_infinite"] = (x, y, z, np.where(np.arange(3000) % 500 == 0, 1e308, h))
    out["h_subnormal"] = (x, y, z, np.where(np.arange(3000) % 2 == 0, 1e-310, h))
    out["h_negative_zero"] = (x, y, z, np.where(np.arange(3000) % 2 == 0, -0.0, h))
    out["h_spread_1e6"] = (x, y, z, h * 10.0 ** rng.uniform(-3, 0.5, 3000))
    out["offset_1e6"] = (x + 1e6, y - 1e6, z + 3e6, h)
    out["scale_2^70"] = (x * 2.0 ** 70, y * 2.0 ** 70, z * 2.0 ** 70, h * 2.0 ** 70)
    out["scale_2^-70"] = (x * 2.0 ** -70, y * 2.0 ** -70, z * 2.0 ** -70, h * 2.0 ** -70)
    out["plane"] = (x, y, np.full(3000, 0.25), h)
    out["line"] = (x, np.full(3000, -1.0), np.full(3000, 2.0), h * 0.1)
    pts = rng.integers(0, 4, size=(3, 2000)).astype(np.float64) * 0.125
    out["coincident_groups"] = (pts[0], pts[1], pts[2], np.full(2000, 1e-3))
    out["all_coincident"] = (np.full(500, 0.3), np.full(500, 0.3), np.full(500, 0.3),
                             np.full(500, 1e-9))
    # ties: x_j = x_i + 2h exactly (not a neighbour) and one ulp inside
    g = np.arange(40, dtype=np.float64) * 0.5
    X, Y, Z = np.meshgrid(g, g[:5], g[:5], indexing="ij")
    out["exact_ties"] = (X.ravel().copy(), Y.ravel().copy(), Z.ravel().copy(),
                         np.full(X.size, 0.25))
    out["ties_inside"] = (X.ravel().copy(), Y.ravel().copy(), Z.ravel().copy(),
                          np.full(X.size, np.nextafter(0.25, 1.0)))
    out["one"] = (np.array([0.5]), np.array([0.5]), np.array([0.5]), np.array([0.1]))
    out["two"] = (np.array([0.0, 1.0]), np.array([0.0, 0.0]), np.array([0.0, 0.0]),
                  np.array([0.5, 0.5000001]))
    return out


@pytest.mark.parametrize("name", sorted(_edge_sets()))
def test_cells_equal_brute_edge_cases(oracle_mod, name):
    x, y, z, h = _edge_sets()[name]
    c = _brute_vs_cells(oracle_mod, x, y, z, h)[0]
    if name == "h_zero":
        assert c.sum() == 0
    if name == "radius_above_diagonal":
        assert np.all(c == len(x))
    if name == "exact_ties":
        assert np.all(c == 1)  # grid spacing 0.5 = 2h exactly: only the point itself
    if name == "ties_inside":
        assert c.max() == 7 and c.min() == 4  # plus its axis neighbours at 0.5 < 2h


def test_cells_empty_set(oracle_mod):
    e = np.zeros(0)
    c, o, nb = oracle_mod.cell_lists(e, e, e, e)
    assert c.shape == (0,) and list(o) == [0] and nb.shape == (0,)
    assert oracle_mod.cell_check(e, e, e, e, np.zeros(0, np.int32), np.zeros(1, np.int64),
                                 np.zeros(0, np.int32))[0] == 0


def test_cells_lattice_every_row_closed_form(oracle_mod):
    """L1M: every row's length from the closed form (93 lattice offsets with
    |v|^2 <= 8, cut at the faces), the total 90 205 144, and symmetry."""
    x, y, z, h = W.lattice()
    c, o, nb = oracle_mod.cell_lists(x, y, z, h)
    m = 100
    i = np.arange(m ** 3)
    ix, iy, iz = i // (m * m), (i // m) % m, i % m
    want = np.zeros(m ** 3, dtype=np.int64)
    offs = [(a, b, cc) for a in range(-2, 3) for b in range(-2, 3) for cc in range(-2, 3)
            if a * a + b * b + cc * cc <= 8]
    assert len(offs) == 93
    for a, b, cc in offs:
        want += ((ix + a >= 0) & (ix + a < m) & (iy + b >= 0) & (iy + b < m) &
                 (iz + cc >= 0) & (iz + cc < m))
    assert np.array_equal(c, want)
    assert o[-1] == 90_205_144
    # each row holds exactly the lattice neighbours of its closed form
    rows = np.repeat(i, c)
    dx = ix[nb] - ix[rows]
    dy = iy[nb] - iy[rows]
    dz = iz[nb] - iz[rows]
    assert np.all(dx * dx + dy * dy + dz * dz <= 8)
    # constant h: j in N(i) <=> i in N(j)
    fwd = rows.astype(np.int64) * m ** 3 + nb
    bwd = nb.astype(np.int64) * m ** 3 + rows
    assert np.array_equal(np.sort(fwd), np.sort(bwd))


def test_cell_check_flags_wrong_rows(oracle_mod):
    x, y, z, h = W.plummer(8000, 4)
    c, o, nb = oracle_mod.lists(x, y, z, h)
    c32 = c.astype(np.int32)
    assert oracle_mod.cell_check(x, y, z, h, c32, o, nb)[0] == 0
    # a changed entry
    nb2 = nb.copy()
    r = 123
    nb2[o[r]] = (nb2[o[r]] + 1) % len(x)
    k, bad = oracle_mod.cell_check(x, y, z, h, c32, o, nb2)
    assert (k, list(bad)) == (1, [r])
    # two rows swapped in length (counts and offsets consistent, content not)
    r2 = 4000
    c3 = c32.copy()
    c3[r2] += 1
    c3[r2 + 1] -= 1
    o3 = np.zeros_like(o)
    np.cumsum(c3, out=o3[1:])
    k, bad = oracle_mod.cell_check(x, y, z, h, c3, o3, nb)
    assert k >= 2 and r2 in bad and r2 + 1 in bad
    # counts inconsistent with offsets
    c4 = c32.copy()
    c4[7] += 1
    assert list(oracle_mod.cell_check(x, y, z, h, c4, o, nb)[1]) == [7]
    # an empty row claimed non-empty
    h5 = h.copy()
    h5[9] = 0.0
    k, bad = oracle_mod.cell_check(x, y, z, h5, c32, o, nb)
    assert 9 in bad


# --------------------------------------------------------------------------
# Planted mistakes: each modified copy of the oracle must fail a pin.
# --------------------------------------------------------------------------

def _mutant(tmp_path, old, new):
    src = open(ORACLE_C).read()
    assert src.count(old) == 1, old
    p = tmp_path / "mut.c"
    p.write_text(src.replace(old, new))
    so = tmp_path / "mut.so"
    subprocess.run(["gcc", "-O2", "-ffp-contract=off", "-fopenmp", "-shared", "-fPIC",
                    "-std=c11", str(p), "-o", str(so), "-lm"], check=True)
    L = ctypes.CDLL(str(so))
    P, I64 = ctypes.c_void_p, ctypes.c_int64
    L.oracle_cell_lists.restype = I64
    L.oracle_cell_lists.argtypes = [P, P, P, P, I64, P, P, P, I64]
    return L


def _mutant_counts(L, x, y, z, h):
    arrs = [np.ascontiguousarray(a, dtype=np.float64) for a in (x, y, z, h)]
    n = len(x)
    c = np.zeros(n, dtype=np.int64)
    o = np.zeros(n + 1, dtype=np.int64)
    L.oracle_cell_lists(*[a.ctypes.data for a in arrs], n, c.ctypes.data, o.ctypes.data,
                        None, 0)
    return c


MUTANTS = {
    "one_cell_fewer_in_x": ("for (int64_t gx = a[0]; gx <= b[0]; ++gx)",
                            "for (int64_t gx = a[0]; gx < b[0]; ++gx)"),
    "range_from_h_not_2h": ("a[k] = cl_cell(q[k] - R, G->o[k], L->c, L->g[k]);",
                            "a[k] = cl_cell(q[k] - hi, G->o[k], L->c, L->g[k]);"),
    "last_z_cell_skipped": ("p < G->n && L->ent[p].key <= k1; ++p) {",
                            "p < G->n && L->ent[p].key < k1; ++p) {"),
    "keys_sorted_on_low_32_bits": ("uint64_t u = ((const cl_ent *)a)->key, v = ((const cl_ent *)b)->key;\n    if (u != v)",
                                   "uint32_t u = ((const cl_ent *)a)->key, v = ((const cl_ent *)b)->key;\n    if (u != v)"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_cell_list_mistakes_fail_a_pin(oracle_mod, tmp_path, name):
    L = _mutant(tmp_path, *MUTANTS[name])
    failed = False
    for seed in range(3):
        x, y, z, h = W.uniform_cube(10_000, seed, 64.0)
        if not np.array_equal(_mutant_counts(L, x, y, z, h), oracle_mod.counts(x, y, z, h)):
            failed = True
            break
    if not failed:
        x, y, z, h = W.plummer(30_000, 5)
        failed = not np.array_equal(_mutant_counts(L, x, y, z, h), oracle_mod.counts(x, y, z, h))
    assert failed, "planted mistake %s was not caught" % name


# --------------------------------------------------------------------------
# Octree option of BuildTree
# --------------------------------------------------------------------------

def _grid4():
    g = np.arange(4) / 3.0
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    return X.ravel().copy(), Y.ravel().copy(), Z.ravel().copy()


def test_octree_hand_built(oracle_mod):
    # 4x4x4 lattice, s = 1: the root splits 2x2x2 into cells of 2x2x2
    # points, each split again into single points: 1 + 8 internal cells,
    # 64 leaves at depth 2.  The b-tree splits once with b = 4 (depth 1).
    t = oracle_mod.build_tree(*_grid4(), s=1, octree=True)
    assert (t.n_internal, t.n_leaves, t.depth, t.b_hist) == (9, 64, 2, {2: 9})
    assert np.all(t.leaf_cnt == 1)
    b = oracle_mod.build_tree(*_grid4(), s=1)
    assert (b.n_internal, b.depth, b.b_hist) == (1, 1, {4: 1})
    # s = 8: one octree split into eight leaves of 8.
    t = oracle_mod.build_tree(*_grid4(), s=8, octree=True)
    assert (t.n_internal, t.n_leaves, t.depth) == (1, 8, 1)
    assert np.all(t.leaf_cnt == 8)


@pytest.mark.parametrize("s", [8, 32, 128])
def test_octree_equals_btree_with_unreachable_ratio(oracle_mod, s):
    x, y, z, _ = W.plummer(40_000, 6)
    o = oracle_mod.build_tree(x, y, z, s=s, octree=True)
    b = oracle_mod.build_tree(x, y, z, s=s, beta=-1.0)
    assert o.b_hist == {2: o.n_internal}
    assert (o.n_internal, o.n_leaves, o.depth, o.max_leaf) == \
           (b.n_internal, b.n_leaves, b.depth, b.max_leaf)
    assert np.array_equal(o.leaf_cnt, b.leaf_cnt)
    assert np.array_equal(o.members, b.members)
    assert o.rounds == 0 and b.rounds > 0


def test_octree_deeper_than_btree(oracle_mod):
    # Section 3.3: on a uniform input the b-tree is one level deep while the
    # octree needs about log8(n / s) levels.
    x, y, z, _ = W.lattice(m=40)
    b = oracle_mod.build_tree(x, y, z, s=64)
    o = oracle_mod.build_tree(x, y, z, s=64, octree=True)
    assert b.depth == 1
    assert o.depth >= 3
    assert np.array_equal(np.sort(o.members), np.arange(len(x)))
